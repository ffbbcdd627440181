// Host-side launch plans of the 3D kernels: which tiles each launch
// covers (single-step fused kernel, two-steps-per-pass kernel and its two
// single-step passes).  Pure integer work, no device code.
#include <algorithm>
#include <functional>
#include <queue>
#include <stdexcept>
#include <vector>

#include "common.hpp"

namespace gem {

// Probes are grouped by (x plane, 4-row band).
int wave3d_ngroups(int nx, int ny) { return nx * ((ny + 3) / 4); }
int wave3d_group_of(int ny, int i, int j) { return i * ((ny + 3) / 4) + j / 4; }

bool wave3d_supported(int nx, int ny, int nz, const Fused3DCfg &c) {
    (void)nx; (void)ny;
    if (!(c.V == 1 || c.V == 2 || c.V == 4)) return false;
    if (c.TX < 0 || c.TX > 4096) return false;
    return nz % c.V == 0;
}

namespace {

struct Range {
    int a, b;
};

// [lo, hi) cut into pieces of at most `w`
void chunks(std::vector<Range> &out, int lo, int hi, int w) {
    for (int a = lo; a < hi; a += w) out.push_back(Range{a, std::min(a + w, hi)});
}

// z segments of [lo, hi) on the grid of multiples of w (w cells per
// segment, lanes below lo or from hi on idle)
struct ZSeg {
    int base, start, end;
};
void zsegs(std::vector<ZSeg> &out, int lo, int hi, int w) {
    if (lo >= hi) return;
    for (int b = lo / w * w; b < hi; b += w) out.push_back(ZSeg{b, std::max(b, lo), std::min(b + w, hi)});
}

}  // namespace

// Launch plan.  x: the planes clear of the x slabs (a tile's plane i0-1
// included) and the slab ends, in chunks of TX planes (TX/4 for the launch
// with x/y CPML code, which has fewer tiles and more latency per plane);
// y: bands of WPB rows (8 interior, 4 slab), clear of the y slabs (row j0-1
// included) or not; z: segments of 64V cells (z-slab cells are handled by
// the correction step of the PZ instances).  The interior launch takes the
// (interior x chunk, interior y band) tiles, the slab launch all others.
// Each launch's tiles run x chunk by x chunk, y bands and z segments
// inside, so that workgroups issued together on one XCD share halo rows;
// each XCD takes a contiguous eighth of the list (padded with empty tiles).
void wave3d_plan(int nx, int ny, int nz, const Fused3DCfg &c, const int *xlohi, const int *ylohi,
                 const int *zlohi, Wave3DPlan &pl) {
    pl.l.clear();
    pl.tiles.clear();
    const int V = c.V;
    const int TX = c.TX > 0 ? c.TX : 16, TXs = std::max(1, TX / 4);
    auto inslab = [](int n, int lo, int hi, int i) { return i >= 0 && i < n && (i < lo || i >= n - hi); };
    const int xl = xlohi[0] == 0 ? 0 : std::min(nx, xlohi[0] + 1);
    const int xh = std::max(xl, nx - xlohi[1]);
    auto add = [&](int Vl, int wpb, bool pxy, bool pz, const std::vector<ZSeg> &zseg) {
        if (zseg.empty()) return;
        const int RB = wpb;
        const int tx = pxy ? TXs : TX;
        Wave3DLaunch l{};
        l.V = Vl;
        l.wpb = wpb;
        l.pxy = pxy;
        l.pz = pz;
        l.off = (int)pl.tiles.size();
        std::vector<Range> xr;
        std::vector<char> xslab;
        auto put = [&](int lo, int hi, bool sl) {
            const size_t n0 = xr.size();
            chunks(xr, lo, hi, tx);
            xslab.resize(xr.size(), sl);
            (void)n0;
        };
        put(0, xl, true);
        put(xl, xh, false);
        put(xh, nx, true);
        // y rows are classified in groups of 8 (the interior band height);
        // the slab launch splits its groups into bands of RB rows
        for (size_t q = 0; q < xr.size(); ++q)
            for (int g0 = 0; g0 < ny; g0 += 8) {
                bool ys = false;
                for (int j = g0 - 1; j < g0 + 8 && j < ny; ++j) ys = ys || inslab(ny, ylohi[0], ylohi[1], j);
                if (pxy != (xslab[q] || ys)) continue;
                for (int j0 = g0; j0 < std::min(g0 + 8, ny); j0 += RB) {
                    const int rows = std::min(RB, ny - j0);
                    const int64_t xn = xr[q].b - xr[q].a;
                    int64_t xs = 0, ysn = 0;
                    for (int i = xr[q].a; i < xr[q].b; ++i) xs += inslab(nx, xlohi[0], xlohi[1], i);
                    for (int j = j0; j < j0 + rows; ++j) ysn += inslab(ny, ylohi[0], ylohi[1], j);
                    for (const ZSeg &z : zseg) {
                        pl.tiles.push_back(Tile3{xr[q].a, xr[q].b, j0, z.base, z.end, z.start, rows, 1});
                        const int64_t zn = z.end - z.start;
                        int64_t zs = 0;
                        for (int k = z.start; k < z.end; ++k) zs += inslab(nz, zlohi[0], zlohi[1], k);
                        l.cells += xn * rows * zn;
                        // four psi per slab a cell lies in
                        l.psi += 4 * (xs * rows * zn + xn * ysn * zn + xn * rows * zs);
                    }
                }
            }
        if (pl.tiles.size() == (size_t)l.off) return;
        while ((pl.tiles.size() - (size_t)l.off) % 8) pl.tiles.push_back(Tile3{0, 0, 0, 0, 0, 0, 0, 0});
        l.n = (int)pl.tiles.size() - l.off;
        pl.l.push_back(l);
    };
    const bool anyxy = xlohi[0] + xlohi[1] + ylohi[0] + ylohi[1] > 0;
    // slab workgroups: 4 rows (fewer registers per wave are left, so smaller
    // workgroups keep more of them resident)
    auto both = [&](int Vl, bool pz, const std::vector<ZSeg> &zseg) {
        add(Vl, 8, false, pz, zseg);
        if (anyxy) add(Vl, 4, true, pz, zseg);
    };
    std::vector<ZSeg> zseg;
    zsegs(zseg, 0, nz, 64 * V);
    both(V, zlohi[0] + zlohi[1] > 0, zseg);
}


bool two3d_supported(int nx, int ny, int nz, int zlo, int zhi) {
    (void)nx; (void)ny;
    if (nz % 4 != 0 || nz > 2 * 64 * 4 || zlo < 0 || zhi < 0 || zlo + zhi > kTwoZMax) return false;
    return ((zlo + 3) & ~3) <= ((nz - zhi) & ~3);
}

int two3d_rows(int nz, bool pz, int mat, bool pxy) {
    const int rz = nz <= 64 * 4 ? 1 : 2;
    return two_waves(pz, mat, pxy) / rz - 2;
}

namespace {

// single-step tiles covering the marked (plane, row) cells of a mask (1 =
// record probes, 2 = do not), full z: per plane, runs of rows with one mark
// in pieces of at most 4 rows; consecutive planes with the same pieces merge
// into x ranges of at most tx planes.
void mask_tiles(const std::vector<unsigned char> &m, int nx, int ny, int nz, int V, int tx, bool pz,
                const int *xlohi, const int *ylohi, const int *zlohi, Wave3DPlan &pl) {
    auto inslab = [](int n, int lo, int hi, int i) { return i >= 0 && i < n && (i < lo || i >= n - hi); };
    struct Piece {
        int j0, n, rec;
        bool operator==(const Piece &o) const { return j0 == o.j0 && n == o.n && rec == o.rec; }
    };
    auto pieces_of = [&](int i) {
        std::vector<Piece> ps;
        int j = 0;
        while (j < ny) {
            const unsigned char mk = m[(size_t)i * ny + j];
            if (!mk) { ++j; continue; }
            int e = j;
            while (e < ny && m[(size_t)i * ny + e] == mk) ++e;
            for (int a = j; a < e; a += 4) ps.push_back(Piece{a, std::min(4, e - a), mk == 1 ? 1 : 0});
            j = e;
        }
        return ps;
    };
    Wave3DLaunch l{};
    l.V = V;
    l.wpb = 4;
    l.pxy = true;
    l.pz = pz;
    l.off = (int)pl.tiles.size();
    const int seg = 64 * V;
    int i = 0;
    while (i < nx) {
        const std::vector<Piece> ps = pieces_of(i);
        int e = i + 1;
        while (e < nx && e - i < tx && pieces_of(e) == ps) ++e;
        int64_t xs = 0;
        for (int a = i; a < e; ++a) xs += inslab(nx, xlohi[0], xlohi[1], a);
        for (const Piece &pc : ps) {
            int64_t ysn = 0;
            for (int b = pc.j0; b < pc.j0 + pc.n; ++b) ysn += inslab(ny, ylohi[0], ylohi[1], b);
            for (int k0 = 0; k0 < nz; k0 += seg) {
                const int k1 = std::min(k0 + seg, nz);
                int64_t zs = 0;
                for (int k = k0; k < k1; ++k) zs += inslab(nz, zlohi[0], zlohi[1], k);
                pl.tiles.push_back(Tile3{i, e, pc.j0, k0, k1, k0, pc.n, pc.rec});
                const int64_t xn = e - i, zn = k1 - k0;
                l.cells += xn * pc.n * zn;
                l.psi += 4 * (xs * pc.n * zn + xn * ysn * zn + xn * pc.n * zs);
            }
        }
        i = e;
    }
    if (pl.tiles.size() == (size_t)l.off) return;
    while ((pl.tiles.size() - (size_t)l.off) % 8) pl.tiles.push_back(Tile3{0, 0, 0, 0, 0, 0, 0, 0});
    l.n = (int)pl.tiles.size() - l.off;
    pl.l.push_back(l);
}

}  // namespace

// x chunk length of the interior two-step tiles when none is given.  Each
// XCD runs its eighth of the list (the widest band group's tiles, x chunk
// by x chunk) in order on its compute units, one workgroup each; a tile
// costs its planes plus two (the planes recomputed at its start), and the
// cost per plane grows slowly with the chunk length (halo rows shared in
// L2 less often).  The chunk (16 .. 128 planes) with the smallest modelled
// finish time is taken; on MI355X the model follows the measured launch
// times within 3 %.
int two3d_auto_tx(int nxi, int nbands, int cus) {
    if (nxi <= 0 || nbands <= 0) return 16;
    const int slots = std::max(1, cus / 8), gb = (nbands + 7) / 8;
    int best = 16;
    double bt = 1e300;
    for (int tx = 16; tx <= std::min(128, std::max(16, nxi)); ++tx) {
        std::priority_queue<double, std::vector<double>, std::greater<double>> q;
        for (int u = 0; u < slots; ++u) q.push(0.0);
        for (int a = 0; a < nxi; a += tx) {
            const int len = std::min(tx, nxi - a);
            for (int b = 0; b < gb; ++b) {
                const double t = q.top();
                q.pop();
                q.push(t + len + 2);
            }
        }
        double mk = 0;
        while (!q.empty()) {
            mk = std::max(mk, q.top());
            q.pop();
        }
        const double t = mk * (1.0 + 0.00052 * (tx - 16));
        if (t < bt - 1e-9) {
            bt = t;
            best = tx;
        }
    }
    return best;
}

void two3d_plan(int nx, int ny, int nz, const Fused3DCfg &c, int mat, bool slab_tb, int txo, int cus,
                const int *xlohi, const int *ylohi, const int *zlohi, TwoPlan &pl) {
    pl.tb.clear();
    pl.tbo.clear();
    pl.tbo_n[0] = pl.tbo_n[1] = 0;
    pl.tb_cells = pl.tb_psi = pl.tbo_cells = pl.tbo_psi = 0;
    pl.pass1.l.clear();
    pl.pass1.tiles.clear();
    pl.pass2.l.clear();
    pl.pass2.tiles.clear();
    const bool pz = zlohi[0] + zlohi[1] > 0;
    const int TX = c.TX > 0 ? c.TX : 16, R = two3d_rows(nz, pz, mat, false);
    pl.slab_tb = slab_tb;
    pl.rows = R;
    pl.rows_o = two3d_rows(nz, pz, mat, true);
    auto inslab = [](int n, int lo, int hi, int i) { return i >= 0 && i < n && (i < lo || i >= n - hi); };
    auto clear = [&](int n, int lo, int hi, int a, int b) {  // no slab cell in [a, b]
        for (int q = std::max(a, 0); q <= std::min(b, n - 1); ++q)
            if (inslab(n, lo, hi, q)) return false;
        return true;
    };
    int64_t zs = 0;
    for (int k = 0; k < nz; ++k) zs += inslab(nz, zlohi[0], zlohi[1], k);
    std::vector<unsigned char> inner((size_t)nx * ny, 0);
    // two-step tiles, x chunk by x chunk, bands inside, over the planes and
    // rows whose cone is clear: [lo + 2, n - hi - 1) of an axis with slabs
    auto range = [](int n, int lo, int hi, int &a, int &b) {
        a = std::min(lo > 0 ? lo + 2 : 0, n);
        b = std::max(hi > 0 ? n - hi - 1 : n, a);
    };
    int xa, xb, ya, yb;
    range(nx, xlohi[0], xlohi[1], xa, xb);
    range(ny, ylohi[0], ylohi[1], ya, yb);
    if (slab_tb) {
        // every cell in two-step tiles.  Launch without x/y-slab code:
        // [xa, xb) in x chunks of TX, [ya, yb) in bands of R rows.  The
        // launch hands each of the 8 XCDs a contiguous eighth of the list,
        // so the bands are split into 8 groups and each group's tiles (x
        // chunk by x chunk, its bands inside) form one eighth, padded to a
        // common length: an XCD's concurrent workgroups are neighbouring
        // bands of one x chunk (their halo rows meet in its L2), and every
        // XCD ends with the short last chunk.
        std::vector<int> bands;
        for (int j0 = ya; j0 < yb; j0 += R) bands.push_back(j0);
        const int nbd = (int)bands.size();
        std::vector<Range> xi, xo;
        pl.tx = c.TX > 0 ? c.TX : two3d_auto_tx(xb - xa, nbd, cus);
        chunks(xi, xa, xb, pl.tx);
        std::vector<std::vector<TileTB>> grp(8);
        for (const Range &c : xi)
            for (int bi = 0; bi < nbd; ++bi) {
                const int j0 = bands[(size_t)bi], nr = std::min(R, yb - j0);
                if (!clear(nx, xlohi[0], xlohi[1], c.a - 2, c.b) || !clear(ny, ylohi[0], ylohi[1], j0 - 2, j0 + nr))
                    throw std::logic_error("two-step plan: interior tile touches a slab");
                grp[(size_t)((int64_t)bi * 8 / nbd)].push_back(TileTB{c.a, c.b, j0, nr});
                pl.tb_cells += (int64_t)(c.b - c.a) * nr * nz;
                pl.tb_psi += 4 * (int64_t)(c.b - c.a) * nr * zs;
            }
        size_t L = 0;
        for (const auto &g : grp) L = std::max(L, g.size());
        for (auto &g : grp) {
            g.resize(L, TileTB{0, 0, 0, 0});
            pl.tb.insert(pl.tb.end(), g.begin(), g.end());
        }
        // launch with it: x chunks of TXo planes over the whole x range,
        // bands of rows_o rows over every row of an x-slab chunk and over
        // [0, ya), [yb, ny) of the others
        const int TXo = txo > 0 ? txo : 16, Ro = pl.rows_o;
        chunks(xo, 0, xa, TXo);
        const size_t nlo = xo.size();
        chunks(xo, xa, xb, TXo);
        const size_t nmid = xo.size();
        chunks(xo, xb, nx, TXo);
        std::vector<TileTB> kind[3];  // cones touching both slab kinds, x slabs only, y slabs only
        for (size_t q = 0; q < xo.size(); ++q) {
            const int i0 = xo[q].a, i1 = xo[q].b;
            int64_t xs = 0;
            for (int i = i0; i < i1; ++i) xs += inslab(nx, xlohi[0], xlohi[1], i);
            auto band = [&](int a, int b) {
                for (int j0 = a; j0 < b; j0 += Ro) {
                    const int nr = std::min(Ro, b - j0);
                    int64_t ysn = 0;
                    for (int jj = j0; jj < j0 + nr; ++jj) ysn += inslab(ny, ylohi[0], ylohi[1], jj);
                    const bool onx = !clear(nx, xlohi[0], xlohi[1], i0 - 2, i1);
                    const bool ony = !clear(ny, ylohi[0], ylohi[1], j0 - 2, j0 + nr);
                    kind[onx && ony ? 0 : (ony ? 2 : 1)].push_back(TileTB{i0, i1, j0, nr});
                    pl.tbo_cells += (int64_t)(i1 - i0) * nr * nz;
                    pl.tbo_psi += 4 * (xs * nr * nz + (int64_t)(i1 - i0) * ysn * nz + (int64_t)(i1 - i0) * nr * zs);
                }
            };
            if (q < nlo || q >= nmid) {
                band(0, ny);
            } else {
                band(0, ya);
                band(yb, ny);
            }
        }
        // the tiles near both slab kinds, then those near one kind: the
        // launch hands each XCD a contiguous eighth of its list, so each
        // eighth takes an eighth of the x-slab tiles and an eighth of the
        // y-slab ones (their chunk lengths differ), padded to a common length
        while (kind[0].size() % 8) kind[0].push_back(TileTB{0, 0, 0, 0});
        pl.tbo = kind[0];
        pl.tbo_n[0] = (int)kind[0].size();
        std::vector<std::vector<TileTB>> part(8);
        size_t Lp = 0;
        for (int e = 0; e < 8; ++e) {
            for (int g = 1; g <= 2; ++g) {
                const size_t n = kind[g].size(), a = n * e / 8, b = n * (e + 1) / 8;
                part[(size_t)e].insert(part[(size_t)e].end(), kind[g].begin() + (long)a, kind[g].begin() + (long)b);
            }
            Lp = std::max(Lp, part[(size_t)e].size());
        }
        for (auto &q : part) {
            q.resize(Lp, TileTB{0, 0, 0, 0});
            pl.tbo.insert(pl.tbo.end(), q.begin(), q.end());
        }
        pl.tbo_n[1] = (int)(8 * Lp);
        while (pl.tb.size() % 8) pl.tb.push_back(TileTB{0, 0, 0, 0});
        return;
    }
    pl.tx = TX;
    for (int i0 = xa; i0 < xb; i0 += TX) {
        const int i1 = std::min(i0 + TX, xb);
        if (!clear(nx, xlohi[0], xlohi[1], i0 - 2, i1)) continue;
        for (int j0 = ya; j0 < yb; j0 += R) {
            const int nr = std::min(R, yb - j0);
            if (!clear(ny, ylohi[0], ylohi[1], j0 - 2, j0 + nr)) continue;
            pl.tb.push_back(TileTB{i0, i1, j0, nr});
            pl.tb_cells += (int64_t)(i1 - i0) * nr * nz;
            pl.tb_psi += 4 * (int64_t)(i1 - i0) * nr * zs;
            for (int i = i0; i < i1; ++i)
                for (int j = j0; j < j0 + nr; ++j) inner[(size_t)i * ny + j] = 1;
        }
    }
    while (pl.tb.size() % 8) pl.tb.push_back(TileTB{0, 0, 0, 0});
    // S: everything else (marked 1); M: its one-cell rim in x and y (marked 2)
    std::vector<unsigned char> s1((size_t)nx * ny, 0), s2((size_t)nx * ny, 0);
    for (size_t q = 0; q < s1.size(); ++q) s1[q] = s2[q] = inner[q] ? 0 : 1;
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            if (!inner[(size_t)i * ny + j]) continue;
            bool near = false;
            for (int a = i - 1; a <= i + 1; ++a)
                for (int b = j - 1; b <= j + 1; ++b)
                    if (a >= 0 && a < nx && b >= 0 && b < ny && !inner[(size_t)a * ny + b]) near = true;
            if (near) s1[(size_t)i * ny + j] = 2;
        }
    const int txs = std::max(1, TX / 4);
    mask_tiles(s1, nx, ny, nz, c.V, txs, pz, xlohi, ylohi, zlohi, pl.pass1);
    mask_tiles(s2, nx, ny, nz, c.V, txs, pz, xlohi, ylohi, zlohi, pl.pass2);
}

}  // namespace gem
