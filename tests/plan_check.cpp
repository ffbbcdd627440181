// Coverage check of the 3D launch plans (host code only; built and run by
// test_plan3d.py).  For random grids, slab widths and tile sizes:
//  * single-step plan: every cell in exactly one tile, tile shapes within the
//    kernel's limits, interior tiles (and their recomputed plane i0-1 and
//    row j0-1) clear of the x/y slabs, z-slab cells only in PZ launches;
//  * two-step plan: the two-step tiles' dependency cones (planes i0-2 .. i1,
//    rows j0-2 .. j0+nrows) clear of the x/y slabs; two-step tiles and the
//    second pass cover every cell exactly once; the first pass covers every
//    cell of the second pass and every (x, y) neighbour of one, once, with
//    probes recorded exactly on the second pass's cells;
//  * 2D multi-step plan: the tiles' own rows and columns cover the grid
//    once; interior tiles' cones (TB rows and the halo lanes' columns around
//    them) clear of the slabs; the default row chunk at measured grids.
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "common.hpp"
using namespace gem;
static bool inslab(int n, int lo, int hi, int i) { return i >= 0 && i < n && (i < lo || i >= n - hi); }
// checks tile shapes of a single-step plan; adds coverage counts (rec: 1 / 0 per cell)
static int walk(const Wave3DPlan &pl, int nx, int ny, int nz, const int *xl, const int *yl, const int *zl,
                std::vector<int> &cov, std::vector<int> &rec) {
    for (auto &l : pl.l) {
        int64_t cells = 0;
        if (l.n % 8) { printf("n not mult of 8\n"); return 1; }
        for (int t = l.off; t < l.off + l.n; ++t) {
            const Tile3 &T = pl.tiles[t];
            if (T.i0 >= T.i1) continue;
            if (T.nrows < 1 || T.nrows > l.wpb || T.j0 + T.nrows > ny) { printf("bad nrows %d wpb %d\n", T.nrows, l.wpb); return 1; }
            if (T.i0 < 0 || T.i1 > nx || T.j0 < 0 || T.j0 >= ny || T.k0 < 0 || T.k1 > nz || T.ks >= T.k1 || T.ks < T.k0) { printf("oob tile\n"); return 1; }
            if (T.k1 - T.k0 > 64 * l.V || (T.k1 - T.ks) % l.V || T.k0 % (l.V * 64) || T.ks % l.V) { printf("bad z seg\n"); return 1; }
            if (T.rec != 0 && T.rec != 1) { printf("bad rec\n"); return 1; }
            for (int i = T.i0 - 1; i < T.i1; ++i)
                if (!l.pxy && inslab(nx, xl[0], xl[1], i)) { printf("interior tile touches x slab i=%d\n", i); return 1; }
            for (int j = T.j0 - 1; j < T.j0 + T.nrows; ++j)
                if (!l.pxy && inslab(ny, yl[0], yl[1], j)) { printf("interior tile touches y slab\n"); return 1; }
            for (int k = T.ks - 1; k < T.k1; ++k)
                if (!l.pz && inslab(nz, zl[0], zl[1], k)) { printf("tile touches z slab without PZ k=%d\n", k); return 1; }
            for (int i = T.i0; i < T.i1; ++i)
                for (int j = T.j0; j < T.j0 + T.nrows; ++j)
                    for (int k = T.ks; k < T.k1; ++k) {
                        const size_t c = ((size_t)i * ny + j) * nz + k;
                        cov[c]++;
                        rec[c] = T.rec;
                        cells++;
                    }
        }
        if (cells != l.cells) { printf("cells mismatch %lld %lld\n", (long long)cells, (long long)l.cells); return 1; }
    }
    return 0;
}
int check1(int nx, int ny, int nz, int V, int TX, const int *xl, const int *yl, const int *zl) {
    Wave3DPlan pl;
    wave3d_plan(nx, ny, nz, Fused3DCfg{V, TX}, xl, yl, zl, pl);
    std::vector<int> cov((size_t)nx * ny * nz, 0), rec(cov.size(), -1);
    if (walk(pl, nx, ny, nz, xl, yl, zl, cov, rec)) return 1;
    for (size_t c = 0; c < cov.size(); ++c)
        if (cov[c] != 1 || rec[c] != 1) { printf("coverage %d rec %d\n", cov[c], rec[c]); return 1; }
    return 0;
}
int check2(int nx, int ny, int nz, int TX, int mat, const int *xl, const int *yl, const int *zl) {
    TwoPlan pl;
    two3d_plan(nx, ny, nz, Fused3DCfg{4, TX}, mat, false, 0, 256, xl, yl, zl, pl);
    const int R = two3d_rows(nz, zl[0] + zl[1] > 0, mat, false);
    if (pl.slab_tb || pl.rows != R || !pl.tbo.empty()) { printf("two-pass plan fields\n"); return 1; }
    std::vector<int> own((size_t)nx * ny, 0);
    if (pl.tb.size() % 8) { printf("tb not mult of 8\n"); return 1; }
    int64_t tbc = 0;
    for (auto &T : pl.tb) {
        if (T.i0 >= T.i1) continue;
        if (T.i0 < 0 || T.i1 > nx || T.j0 < 0 || T.nrows < 1 || T.nrows > R || T.j0 + T.nrows > ny) { printf("bad tb tile\n"); return 1; }
        for (int i = T.i0 - 2; i <= T.i1; ++i)
            if (inslab(nx, xl[0], xl[1], i)) { printf("tb cone touches x slab\n"); return 1; }
        for (int j = T.j0 - 2; j <= T.j0 + T.nrows; ++j)
            if (inslab(ny, yl[0], yl[1], j)) { printf("tb cone touches y slab\n"); return 1; }
        for (int i = T.i0; i < T.i1; ++i)
            for (int j = T.j0; j < T.j0 + T.nrows; ++j) { own[(size_t)i * ny + j]++; tbc += nz; }
    }
    if (tbc != pl.tb_cells) { printf("tb cells mismatch\n"); return 1; }
    std::vector<int> c1((size_t)nx * ny * nz, 0), r1(c1.size(), -1), c2(c1.size(), 0), r2(c1.size(), -1);
    if (walk(pl.pass1, nx, ny, nz, xl, yl, zl, c1, r1)) return 1;
    if (walk(pl.pass2, nx, ny, nz, xl, yl, zl, c2, r2)) return 1;
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            const int o = own[(size_t)i * ny + j];
            if (o > 1) { printf("tb overlap\n"); return 1; }
            bool needed = o == 0;  // S cell itself
            for (int a = i - 1; a <= i + 1; ++a)
                for (int b = j - 1; b <= j + 1; ++b)
                    if (a >= 0 && a < nx && b >= 0 && b < ny && own[(size_t)a * ny + b] == 0) needed = true;
            for (int k = 0; k < nz; ++k) {
                const size_t c = ((size_t)i * ny + j) * nz + k;
                if (o + c2[c] != 1) { printf("final coverage %d+%d at %d %d %d\n", o, c2[c], i, j, k); return 1; }
                if (c2[c] && r2[c] != 1) { printf("pass2 rec\n"); return 1; }
                if (c1[c] > 1) { printf("pass1 overlap\n"); return 1; }
                if (needed && c1[c] != 1) { printf("pass1 misses a needed cell %d %d %d\n", i, j, k); return 1; }
                if (c1[c] && r1[c] != (o == 0 ? 1 : 0)) { printf("pass1 rec wrong\n"); return 1; }
            }
        }
    return 0;
}
// two-step plan with the slab tiles in the two-step kernel: the interior
// list's tiles have a cone clear of the x/y slabs and at most R rows, the
// slab list's at most rows_o rows and txo planes (TX inside [lo+2, n-hi-1));
// together they own every (i, j) once; no single-step passes
int check2s(int nx, int ny, int nz, int TX, int txo, int mat, const int *xl, const int *yl, const int *zl) {
    TwoPlan pl;
    two3d_plan(nx, ny, nz, Fused3DCfg{4, TX}, mat, true, txo, 256, xl, yl, zl, pl);
    const bool pz = zl[0] + zl[1] > 0;
    const int R = two3d_rows(nz, pz, mat, false), Ro = two3d_rows(nz, pz, mat, true);
    const int tx = TX > 0 ? TX : pl.tx, txs = txo > 0 ? txo : 16;
    if (TX > 0 && pl.tx != TX) { printf("slab plan tx\n"); return 1; }
    if (TX == 0 && (pl.tx < 16 || pl.tx > 128)) { printf("auto tx %d\n", pl.tx); return 1; }
    if (!pl.slab_tb || pl.rows != R || pl.rows_o != Ro || !pl.pass1.l.empty() || !pl.pass2.l.empty()) {
        printf("slab plan fields\n");
        return 1;
    }
    if (pl.tb.size() % 8 || pl.tbo.size() % 8) { printf("slab plan lists not mult of 8\n"); return 1; }
    // slab list in two groups (cones touching both slab kinds, then one
    // kind), each a multiple of 8: the second group's kernel holds a code
    // path per kind, without the other kind's psi code
    if (pl.tbo_n[0] + pl.tbo_n[1] != (int)pl.tbo.size() || pl.tbo_n[0] % 8 || pl.tbo_n[1] % 8) {
        printf("slab groups\n");
        return 1;
    }
    for (size_t q = 0; q < pl.tbo.size(); ++q) {
        const TileTB &T = pl.tbo[q];
        if (T.i0 >= T.i1) continue;
        const bool both = q < (size_t)pl.tbo_n[0];
        bool onx = false, ony = false;
        for (int i = T.i0 - 2; i <= T.i1; ++i) onx = onx || inslab(nx, xl[0], xl[1], i);
        for (int j = T.j0 - 2; j <= T.j0 + T.nrows; ++j) ony = ony || inslab(ny, yl[0], yl[1], j);
        // the kernel's test of the kind: planes [i0-2, i1] clipped to the grid
        const int a = std::max(T.i0 - 2, 0), b = std::min(T.i1, nx - 1);
        const bool kx = (xl[0] > 0 && a < xl[0]) || (xl[1] > 0 && b >= nx - xl[1]);
        if ((both && !(onx && ony)) || (!both && (onx == ony || kx != onx))) {
            printf("slab group of tile %d\n", (int)q);
            return 1;
        }
    }
    std::vector<int> own((size_t)nx * ny, 0);
    int64_t zs = 0;
    for (int k = 0; k < nz; ++k) zs += inslab(nz, zl[0], zl[1], k);
    for (int list = 0; list < 2; ++list) {
        int64_t cells = 0, psi = 0;
        for (const TileTB &T : list ? pl.tbo : pl.tb) {
            if (T.i0 >= T.i1) continue;
            if (T.i0 < 0 || T.i1 > nx || T.j0 < 0 || T.nrows < 1 || T.j0 + T.nrows > ny ||
                T.nrows > (list ? Ro : R) || T.i1 - T.i0 > std::max(tx, txs)) {
                printf("bad slab-plan tile list %d\n", list);
                return 1;
            }
            if (list == 0) {
                for (int i = T.i0 - 2; i <= T.i1; ++i)
                    if (inslab(nx, xl[0], xl[1], i)) { printf("interior cone touches x slab\n"); return 1; }
                for (int j = T.j0 - 2; j <= T.j0 + T.nrows; ++j)
                    if (inslab(ny, yl[0], yl[1], j)) { printf("interior cone touches y slab\n"); return 1; }
            }
            for (int i = T.i0; i < T.i1; ++i)
                for (int j = T.j0; j < T.j0 + T.nrows; ++j) {
                    own[(size_t)i * ny + j]++;
                    cells += nz;
                    psi += 4 * ((inslab(nx, xl[0], xl[1], i) + inslab(ny, yl[0], yl[1], j)) * (int64_t)nz + zs);
                }
        }
        if (cells != (list ? pl.tbo_cells : pl.tb_cells) || psi != (list ? pl.tbo_psi : pl.tb_psi)) {
            printf("slab plan counts list %d\n", list);
            return 1;
        }
    }
    for (int o : own)
        if (o != 1) { printf("slab plan coverage %d\n", o); return 1; }
    return 0;
}
// 2D multi-step plan: own columns [ja, ja + own) and rows [i0, i1) of the
// tiles cover the grid once; interior tiles' cones clear of the slabs
int check2d(int nx, int ny, int V, int TB, int TX, int TXo, const int *xl, const int *yl) {
    std::vector<Tile2T> in, out;
    tb2d_plan(7, nx, ny, V, TB, TX, TXo, xl, yl, in, out);
    std::vector<int> cov((size_t)nx * ny, 0);
    const int ow = tb2d_own(V, TB), hw = tb2d_halo(V, TB) * V;
    for (int pass = 0; pass < 2; ++pass)
        for (const Tile2T &t : pass ? out : in) {
            if (t.prob != 7 || t.i0 < 0 || t.i1 > nx || t.i0 >= t.i1 || t.i1 - t.i0 > (pass && TXo > 0 ? TXo : TX) ||
                t.ja < 0 || t.ja >= ny ||
                t.ja % V) {
                printf("bad 2d tile\n");
                return 1;
            }
            if (pass == 0) {
                for (int i = t.i0 - TB; i < t.i1 + TB; ++i)
                    if (inslab(nx, xl[0], xl[1], i)) { printf("2d interior cone touches x slab\n"); return 1; }
                for (int j = t.ja - hw; j < t.ja - hw + 64 * V; ++j)
                    if (inslab(ny, yl[0], yl[1], j)) { printf("2d interior cone touches y slab\n"); return 1; }
            }
            for (int i = t.i0; i < t.i1; ++i)
                for (int j = t.ja; j < std::min(ny, t.ja + ow); ++j) cov[(size_t)i * ny + j]++;
        }
    for (int c : cov)
        if (c != 1) { printf("2d coverage %d\n", c); return 1; }
    return 0;
}

int main(int argc, char **argv) {
    // argv[1]: divide the random case counts (a shorter run under sanitizers)
    const int div = argc > 1 ? std::max(1, atoi(argv[1])) : 1;
    int bad = 0, n = 0;
    // two-step support rule: nz % 4, nz <= 512, at most 64 slab cells, no
    // 4-cell group with cells of both z slabs
    const struct { int nz, lo, hi; bool ok; } sup[] = {
        {512, 12, 12, true}, {516, 12, 12, false}, {510, 12, 12, false}, {256, 0, 0, true},
        {128, 40, 24, true}, {128, 40, 25, false}, {12, 5, 5, false}, {16, 6, 7, true}, {16, 7, 7, true}, {16, 9, 6, false}};
    for (const auto &c : sup)
        if (two3d_supported(8, 8, c.nz, c.lo, c.hi) != c.ok) {
            printf("two3d_supported(%d, %d, %d) wrong\n", c.nz, c.lo, c.hi);
            ++bad;
        }
    // default row chunk of the 2D four-step pass on 256 CUs, at the grids it
    // was measured on (V = 2: the chunk whose interior workgroups number 4-5
    // per CU, else 8; V = 1: 32 rows with 4 per CU, else the longest with 2
    // per CU, else 4)
    const struct { int n, V, tx; } dtx[] = {
        {4096, 2, 32}, {3072, 2, 16}, {6400, 2, 8}, {2048, 2, 8}, {6400, 1, 32}, {4096, 1, 32}, {3000, 1, 32},
        {2048, 1, 16}, {1448, 1, 16}, {1024, 1, 8}, {256, 1, 4}};
    for (const auto &c : dtx)
        if (tb2d_default_tx(c.n, c.n, c.V, 256) != c.tx) {
            printf("tb2d_default_tx(%d, V %d) = %d, expected %d\n", c.n, c.V, tb2d_default_tx(c.n, c.n, c.V, 256), c.tx);
            ++bad;
        }
    srand(1);
    for (int t = 0; t < 3000 / div; ++t) {
        int V = 1 << (rand() % 3);
        int nx = 1 + rand() % 40, ny = 1 + rand() % 90, nz = V * (1 + rand() % 100);
        int TX = rand() % 3 == 0 ? 0 : 1 + rand() % 20;
        int s[6];
        for (int q = 0; q < 6; ++q) s[q] = rand() % 3 == 0 ? 0 : rand() % 15;
        if (s[0] + s[1] > nx) s[0] = s[1] = 0;
        if (s[2] + s[3] > ny) s[2] = s[3] = 0;
        if (s[4] + s[5] > nz) s[4] = s[5] = 0;
        int r = check1(nx, ny, nz, V, TX, s, s + 2, s + 4);
        if (r) printf("  single case nx %d ny %d nz %d V %d TX %d s %d %d %d %d %d %d\n", nx, ny, nz, V, TX, s[0], s[1], s[2], s[3], s[4], s[5]);
        bad += r; ++n;
        // two-step plan: nz multiple of 4, <= 512, z slabs <= 64
        int nz2 = 4 * (1 + rand() % 128);
        if (s[4] + s[5] > nz2 || s[4] + s[5] > 64) s[4] = s[5] = 0;
        const int mat = rand() % 3;
        r = check2(nx, ny, nz2, TX, mat, s, s + 2, s + 4);
        if (r) printf("  two case nx %d ny %d nz %d TX %d mat %d s %d %d %d %d %d %d\n", nx, ny, nz2, TX, mat, s[0], s[1], s[2], s[3], s[4], s[5]);
        bad += r; ++n;
        const int txo = rand() % 3 == 0 ? 0 : 1 + rand() % 20;
        r = check2s(nx, ny, nz2, TX, txo, mat, s, s + 2, s + 4);
        if (r) printf("  slab-tb case nx %d ny %d nz %d TX %d txo %d mat %d s %d %d %d %d %d %d\n", nx, ny, nz2, TX, txo, mat, s[0], s[1], s[2], s[3], s[4], s[5]);
        bad += r; ++n;
    }
    for (int t = 0; t < 2000 / div; ++t) {
        const int V = 1 << (rand() % 3), TB = rand() % 2 ? 2 : 4;
        const int nx = 1 + rand() % 300, ny = V * (1 + rand() % 200), TX = 1 + rand() % 40;
        int s[4];
        for (int q = 0; q < 4; ++q) s[q] = rand() % 3 == 0 ? 0 : rand() % 20;
        if (s[0] + s[1] >= nx) s[0] = s[1] = 0;
        if (s[2] + s[3] >= ny) s[2] = s[3] = 0;
        const int TXo = rand() % 3 == 0 ? 0 : 1 + rand() % 10;
        const int r = check2d(nx, ny, V, TB, TX, TXo, s, s + 2);
        if (r) printf("  2d case nx %d ny %d V %d TB %d TX %d TXo %d s %d %d %d %d\n", nx, ny, V, TB, TX, TXo, s[0], s[1], s[2], s[3]);
        bad += r;
    }
    printf("%d / %d bad\n", bad, n);
    return bad != 0;
}
