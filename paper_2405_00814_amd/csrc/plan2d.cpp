// Host-side tile plan of the 2D multi-step kernel (pure integer work).
#include <algorithm>
#include <vector>

#include "common.hpp"

namespace gem {

bool tb2d_supported(int ny, int V, int TB, int TX) {
    if (!(V == 1 || V == 2 || V == 4) || !(TB == 2 || TB == 4)) return false;
    if (TX < 1 || TX > 65536) return false;
    return ny % V == 0;
}

// The default row chunk.  Measured on 1448^2 - 6400^2 dielectric grids
// (four steps per pass, CPML tiles on a second stream, one column per lane):
// 32-row chunks where the interior workgroups (four strips each) still
// number at least 4 per CU, else 16 where they number 2 per CU, else 8 or
// 4 (4096^2: 373 Gcell/s at 32 rows, 376 at 16; 6400^2: 454 vs 412;
// 3000^2: 334 vs 317; 2048^2: 16 rows, 234 vs 214).  With two columns per
// lane: 32 rows where the interior workgroups number 4-5 per CU, 16 in
// that band, else 8.
int tb2d_default_tx(int nx, int ny, int V, int cus) {
    const int own = tb2d_own(V, 4);
    auto wgs = [&](int tx) { return (int64_t)((nx + tx - 1) / tx) * ((ny + own - 1) / own) / 4; };
    if (V == 2) {
        for (int tx : {32, 16})
            if (wgs(tx) >= 4 * (int64_t)cus && wgs(tx) <= 5 * (int64_t)cus) return tx;
        return 8;
    }
    if (wgs(32) >= 4 * (int64_t)cus) return 32;
    for (int tx : {16, 8})
        if (wgs(tx) >= 2 * (int64_t)cus) return tx;
    return 4;
}

void tb2d_plan(int prob, int nx, int ny, int V, int TB, int TX, int TXo, const int *xlohi, const int *ylohi,
               std::vector<Tile2T> &inner, std::vector<Tile2T> &outer) {
    if (TXo < 1) TXo = TX;
    const int ow = tb2d_own(V, TB), hw = tb2d_halo(V, TB) * V;
    auto clear = [](int n, int lo, int hi, int a, int b) {  // no slab index in [a, b)
        a = std::max(a, 0);
        b = std::min(b, n);
        for (int q = a; q < b; ++q)
            if (q < lo || q >= n - hi) return false;
        return true;
    };
    for (int i0 = 0; i0 < nx; i0 += TX) {
        const int i1 = std::min(i0 + TX, nx);
        const bool xc = clear(nx, xlohi[0], xlohi[1], i0 - TB, i1 + TB);
        for (int ja = 0; ja < ny; ja += ow) {
            const bool yc = clear(ny, ylohi[0], ylohi[1], ja - hw, ja - hw + 64 * V);
            if (xc && yc) {
                inner.push_back(Tile2T{prob, i0, i1, ja});
            } else {
                // tiles with the CPML code in pieces of TXo rows
                for (int a = i0; a < i1; a += TXo) outer.push_back(Tile2T{prob, a, std::min(a + TXo, i1), ja});
            }
        }
    }
}

}  // namespace gem
