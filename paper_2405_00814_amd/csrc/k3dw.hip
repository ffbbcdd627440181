// Fused single-pass 3D Yee step (H layer, then E layer, CPML, source and
// probes in one kernel).  No LDS and no block barriers.
//
// A thread owns V consecutive z cells of one y row and marches through the
// x planes i0 .. i1-1 of its tile.  At plane i it writes H^{n+1/2} and
// E^{n+1} of its cells.  The E layer needs H of the neighbours at i-1, j-1
// and k-1:
//   i-1: the thread's own H of the previous plane, carried in registers
//        (recomputed from the old state for the first plane of the tile);
//   j-1: recomputed from the old state of row j-1 (that row is the
//        neighbouring wavefront's own data and comes from the caches);
//   k-1: the previous element of the vector, a lane shuffle, or (first
//        active lane of a z segment) recomputed at z = ks-1.
// The H layer needs E at i+1 (loaded once and carried to the next plane as
// the own E), at j+1 and at k+1 (the next element, a shuffle or, for the
// segment's last lane, a load).  State is double buffered (read s0, write
// s1), so every recomputed value equals its owner's value (up to the
// rounding of the same arithmetic written in another place).
//
// Tiles: (x range, band of WPB y rows, z segment of 64*V cells).  Rows
// of one workgroup exchange the values their neighbours need through LDS
// (old Ex, Ez for the row below; new Hx, Hz for the row above), so only the
// band's first row recomputes H at j-1 and only its last loads E at j+1.  The
// interior tiles (no x or y CPML slab touched) run an instance without the
// x/y CPML code, the others one with it.  z-slab cells are lanes of the same
// segments: the main formulas take the interior profile and the lanes with
// slab cells add the CPML terms in a correction step.
#include "common.hpp"
#include "devutil.hpp"
#include "k3dcell.hpp"

namespace gem {

// MAT: 0 = Cb map only, 1 = Ca and Cb maps, 2 = Ca, Cb and Db maps.
// PXY: CPML code for the x and y slabs; PZ: for the z slabs.  A tile whose
// cells and recomputed neighbours (plane i0-1, row j-1, z = ks-1) touch no x
// or y slab may run PXY = false, none touching a z slab PZ = false.
// WPB: wavefronts per workgroup, one y row each
template <int V, int WPB, bool PXY, bool PZ, int MAT>
__global__ __launch_bounds__(64 * WPB) void k3d_march(Prob3D p, const Tile3 *tiles, ProbeTiles pt,
                                                 int64_t step) {
    constexpr int LZ = 64;  // lanes per z row
    const Tile3 T = tiles[xcd_block(blockIdx.x, gridDim.x)];
    if (T.i0 >= T.i1) return;  // padding
    const int lane = threadIdx.x & 63;
    const int zlane = lane;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int rw = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // row of the band
    const int j = T.j0 + rw;  // wave-uniform
    // z segment: lanes from the aligned base T.k0, active on [ks, kend)
    const int ks = T.ks, kend = T.k1, kb = T.k0 + zlane * V, km = ks - 1;
    const bool ok = rw < T.nrows && kb >= ks && kb < kend;  // ks, kend: multiples of V
    const bool first = kb == ks;
    const bool yj = j + 1 < ny, jm = j >= 1;
    const bool ke = kend < nz;
    const bool last = kb + V == kend;  // lane 63 unless the segment is cut short
    const unsigned sxs = (unsigned)ny * nz, sys = nz;
    const int jr = rw < T.nrows ? j : T.j0;
    const int sy = p.y.lo + p.y.hi, sz = p.z.lo + p.z.hi;
    const float *ex0 = p.s0.f[FDTD_EX], *ey0 = p.s0.f[FDTD_EY], *ez0 = p.s0.f[FDTD_EZ];
    const float *hx0 = p.s0.f[FDTD_HX], *hy0 = p.s0.f[FDTD_HY], *hz0 = p.s0.f[FDTD_HZ];
    float *const *P0 = p.s0.psi;
    float *const *P1 = p.s1.psi;
    auto zero = [](float (&a)[V]) {
#pragma unroll
        for (int v = 0; v < V; ++v) a[v] = 0.f;
    };
    auto ld = [&](float (&a)[V], const float *base, unsigned off, bool cond) {
        if (cond) ldv<V>(a, base + off);
        else zero(a);
    };
    // z slabs: the main formulas use the interior 1/dz (kappa = 1 outside the
    // slabs); cells of a lane inside a z slab then add (1/(kappa dz) - 1/dz) D
    // and their psi term in a correction step (divergent, lanes with slab
    // cells only)
    int zsv[V];  // z-slab index of cell kb+v (-1 outside, or without z slabs)
    bool zany = false;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        zsv[v] = (PZ && ok) ? slab_index(p.z, kb + v) : -1;
        zany = zany || zsv[v] >= 0;
    }
    const float idzH = p.z.kH[p.z.lo], idzE = p.z.kE[p.z.lo];  // index lo: first one outside
    // the old z-slab psi a[q] of the lane's slab cells and b, c, 1/(kappa dz)
    // of the H or E profile (elements outside the slab read a[row])
    auto zload = [&](float (&o)[V], float (&kk)[V], float (&bb)[V], float (&cc)[V], const float *a,
                     unsigned row, const float *kt, const float *bt, const float *ct) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            o[v] = a[row + (zsv[v] >= 0 ? zsv[v] : 0)];
            kk[v] = kt[kb + v];
            bb[v] = bt[kb + v];
            cc[v] = ct[kb + v];
        }
    };

    // y profiles (wave-uniform)
    const AxP Y = axp<PXY>(p.y, jr), Ym = axp<PXY>(p.y, jm && j < ny ? j - 1 : 0);

    // carried between planes: E (y, z) of the current plane and H (y, z) of
    // the previous one
    float eyc[V], ezc[V], hyp[V], hzp[V];
    {
        const int i = T.i0;
        const unsigned r0 = ((unsigned)i * ny + jr) * nz, c = r0 + kb;
        ld(eyc, ey0, c, ok);
        ld(ezc, ez0, c, ok);
        // ---- Hy, Hz at (i0-1, j) from the old state ----
        zero(hyp);
        zero(hzp);
        if (i >= 1) {  // uniform over the workgroup
            const bool o = ok;
            const unsigned q0 = c - sxs;
            const AxP Xm = axp<PXY>(p.x, i - 1);
            float aex[V], aey[V], aez[V], aexy[V], ahy[V], ahz[V], adb[V];
            ld(aex, ex0, q0, o);
            ld(aey, ey0, q0, o);
            ld(aez, ez0, q0, o);
            ld(aexy, ex0, q0 + sys, o && yj);
            ld(ahy, hy0, q0, o);
            ld(ahz, hz0, q0, o);
#pragma unroll
            for (int v = 0; v < V; ++v) adb[v] = p.db0;
            if (MAT == 2 && o) ldv<V>(adb, p.db + q0);
            const float aex_e = (o && last && ke) ? ex0[r0 - sxs + kend] : 0.f;
            float pyx[V], pzx[V], pzy[V], dExzA[V];
            const bool inx = PXY && o && Xm.s >= 0, iny = PXY && o && Y.s >= 0;
            const unsigned qx = inx ? xs3(Xm.s, j, kb, ny, nz) : 0, qy = iny ? ys3(i - 1, Y.s, kb, sy, nz) : 0;
            ld(pyx, P0[PSI_HYX], qx, inx);
            ld(pzx, P0[PSI_HZX], qx, inx);
            ld(pzy, P0[PSI_HZY], qy, iny);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const float dExz = znext<V>(aex, v, aex_e, last) - aex[v];
                const float dEzx = ezc[v] - aez[v];
                const float dEyx = eyc[v] - aey[v];
                const float dExy = aexy[v] - aex[v];
                dExzA[v] = dExz;
                const float vyx = inx ? Xm.bH * pyx[v] + Xm.cH * dEzx : 0.f;
                const float vzx = inx ? Xm.bH * pzx[v] + Xm.cH * dEyx : 0.f;
                const float vzy = iny ? Y.bH * pzy[v] + Y.cH * dExy : 0.f;
                if (o) {
                    hyp[v] = ahy[v] - adb[v] * ((idzH * dExz) - (Xm.kH * dEzx + vyx));
                    hzp[v] = ahz[v] - adb[v] * ((Xm.kH * dEyx + vzx) - (Y.kH * dExy + vzy));
                }
            }
            if (PZ && zany) {
                float oz[V], kh[V], bh[V], chh[V];
                zload(oz, kh, bh, chh, P0[PSI_HYZ], zs3(i - 1, j, 0, ny, sz), p.z.kH, p.z.bH, p.z.cH);
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if (zsv[v] >= 0) {
                        const float pyz = bh[v] * oz[v] + chh[v] * dExzA[v];
                        hyp[v] -= adb[v] * ((kh[v] - idzH) * dExzA[v] + pyz);
                    }
            }
        }
    }

    // LDS rows: [0] Ex, [1] Ez (old), [2] Hx, [3] Hz (new) of every thread's
    // V cells at index threadIdx.x * V; the row above is LZ threads back
    __shared__ float sh[4][WPB * 64 * V];
    const int tq = (int)threadIdx.x * V;
    const bool top = rw == 0, bot = rw == T.nrows - 1;  // first and last row of the band
    for (int i = T.i0; i < T.i1; ++i) {
        const bool xi = i + 1 < nx, im = i >= 1;
        const unsigned r0 = ((unsigned)i * ny + jr) * nz;  // row (i, j)
        const unsigned c = r0 + kb;
        const AxP X = axp<PXY>(p.x, i);

        // ---- E and H at the own cells; E at (i+1), (j+1) ----
        float ex[V], ey[V], ez[V], ey_x[V], ez_x[V], ex_y[V], ez_y[V], hxo[V], hyo[V], hzo[V];
        float db[V], cb[V], ca[V];
#pragma unroll
        for (int v = 0; v < V; ++v) { ey[v] = eyc[v]; ez[v] = ezc[v]; }
        ld(ex, ex0, c, ok);
        ld(ey_x, ey0, c + sxs, ok && xi);
        ld(ez_x, ez0, c + sxs, ok && xi);
        ld(ex_y, ex0, c + sys, ok && yj && bot);  // other rows: from LDS below
        ld(ez_y, ez0, c + sys, ok && yj && bot);
        ld(hxo, hx0, c, ok);
        ld(hyo, hy0, c, ok);
        ld(hzo, hz0, c, ok);
        ld(cb, p.cb, c, ok);
#pragma unroll
        for (int v = 0; v < V; ++v) { ca[v] = 1.f; db[v] = p.db0; }
        if (MAT >= 1 && ok) ldv<V>(ca, p.ca + c);
        if (MAT == 2 && ok) ldv<V>(db, p.db + c);
        const bool s63 = ok && last && ke;
        const float ey_e = s63 ? ey0[r0 + kend] : 0.f;
        const float ex_e = s63 ? ex0[r0 + kend] : 0.f;
        // old z-slab psi of the lane's slab cells, issued with the field loads
        float zo[4][V];
        const unsigned zrow = zs3(i, j, 0, ny, sz);
        if (PZ && zany) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const unsigned q = zrow + (zsv[v] >= 0 ? zsv[v] : 0);
                zo[0][v] = P0[PSI_HXZ][q];
                zo[1][v] = P0[PSI_HYZ][q];
                zo[2][v] = P0[PSI_EXZ][q];
                zo[3][v] = P0[PSI_EYZ][q];
            }
        }
        // x/y-slab psi of H (vector rows), also issued before the barrier
        float pxy[V], pzx[V], pyx[V], pzy[V];
        const bool iny = PXY && ok && Y.s >= 0, inx = PXY && ok && X.s >= 0;
        const unsigned qy = iny ? ys3(i, Y.s, kb, sy, nz) : 0, qx = inx ? xs3(X.s, j, kb, ny, nz) : 0;
        ld(pxy, P0[PSI_HXY], qy, iny);
        ld(pzy, P0[PSI_HZY], qy, iny);
        ld(pyx, P0[PSI_HYX], qx, inx);
        ld(pzx, P0[PSI_HZX], qx, inx);
        stv<V>(&sh[0][tq], ex);
        stv<V>(&sh[1][tq], ez);
        __syncthreads();
        if (!bot && ok && yj) {
            ldv<V>(ex_y, &sh[0][tq + LZ * V]);
            ldv<V>(ez_y, &sh[1][tq + LZ * V]);
        }

        // ---- H layer at the own cells ----
        float hx[V], hy[V], hz[V];
        {
            float dEyzA[V], dExzA[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const float dEzy = ez_y[v] - ez[v];
                const float dEyz = znext<V>(ey, v, ey_e, last) - ey[v];
                const float dExz = znext<V>(ex, v, ex_e, last) - ex[v];
                const float dEzx = ez_x[v] - ez[v];
                const float dEyx = ey_x[v] - ey[v];
                const float dExy = ex_y[v] - ex[v];
                dEyzA[v] = dEyz;
                dExzA[v] = dExz;
                if (iny) { pxy[v] = Y.bH * pxy[v] + Y.cH * dEzy; pzy[v] = Y.bH * pzy[v] + Y.cH * dExy; }
                if (inx) { pyx[v] = X.bH * pyx[v] + X.cH * dEzx; pzx[v] = X.bH * pzx[v] + X.cH * dEyx; }
                hx[v] = hxo[v] - db[v] * ((Y.kH * dEzy + (iny ? pxy[v] : 0.f)) - (idzH * dEyz));
                hy[v] = hyo[v] - db[v] * ((idzH * dExz) - (X.kH * dEzx + (inx ? pyx[v] : 0.f)));
                hz[v] = hzo[v] - db[v] * ((X.kH * dEyx + (inx ? pzx[v] : 0.f)) - (Y.kH * dExy + (iny ? pzy[v] : 0.f)));
            }
            if (PZ && zany) {
                const unsigned row = zrow;
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if (zsv[v] >= 0) {
                        const float kh = p.z.kH[kb + v], bh = p.z.bH[kb + v], chh = p.z.cH[kb + v];
                        const float pxz = bh * zo[0][v] + chh * dEyzA[v];
                        const float pyz = bh * zo[1][v] + chh * dExzA[v];
                        P1[PSI_HXZ][row + zsv[v]] = pxz;
                        P1[PSI_HYZ][row + zsv[v]] = pyz;
                        hx[v] += db[v] * ((kh - idzH) * dEyzA[v] + pxz);
                        hy[v] -= db[v] * ((kh - idzH) * dExzA[v] + pyz);
                    }
            }
            if (iny) { stv<V>(P1[PSI_HXY] + qy, pxy); stv<V>(P1[PSI_HZY] + qy, pzy); }
            if (inx) { stv<V>(P1[PSI_HYX] + qx, pyx); stv<V>(P1[PSI_HZX] + qx, pzx); }
        }

        // ---- Hx, Hz at (i, j-1): from LDS, or (first row of the band)
        // recomputed from the old state ----
        float hx_jm[V], hz_jm[V];
        zero(hx_jm);
        zero(hz_jm);
        stv<V>(&sh[2][tq], hx);
        stv<V>(&sh[3][tq], hz);
        __syncthreads();
        if (!top && ok && jm) {
            ldv<V>(hx_jm, &sh[2][tq - LZ * V]);
            ldv<V>(hz_jm, &sh[3][tq - LZ * V]);
        }
        if (top) {  // wave-uniform
            const bool o = ok && jm && top;
            const unsigned q0 = c - (jm ? sys : 0u);
            float aex[V], aey[V], aez[V], aeyx[V], ahx[V], ahz[V], adb[V];
            ld(aex, ex0, q0, o);
            ld(aey, ey0, q0, o);
            ld(aez, ez0, q0, o);
            ld(aeyx, ey0, q0 + sxs, o && xi);
            ld(ahx, hx0, q0, o);
            ld(ahz, hz0, q0, o);
#pragma unroll
            for (int v = 0; v < V; ++v) adb[v] = p.db0;
            if (MAT == 2 && o) ldv<V>(adb, p.db + q0);
            const float aey_e = (o && last && ke) ? ey0[r0 - sys + kend] : 0.f;
            float pxy[V], pzy[V], pzx[V];
            const bool iny = PXY && o && Ym.s >= 0, inx = PXY && o && X.s >= 0;
            const unsigned qy = iny ? ys3(i, Ym.s, kb, sy, nz) : 0, qx = inx ? xs3(X.s, j - 1, kb, ny, nz) : 0;
            ld(pxy, P0[PSI_HXY], qy, iny);
            ld(pzy, P0[PSI_HZY], qy, iny);
            ld(pzx, P0[PSI_HZX], qx, inx);
            float dEyzB[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const float dEzy = ez[v] - aez[v];
                const float dEyz = znext<V>(aey, v, aey_e, last) - aey[v];
                const float dEyx = aeyx[v] - aey[v];
                const float dExy = ex[v] - aex[v];
                dEyzB[v] = dEyz;
                const float vxy = iny ? Ym.bH * pxy[v] + Ym.cH * dEzy : 0.f;
                const float vzy = iny ? Ym.bH * pzy[v] + Ym.cH * dExy : 0.f;
                const float vzx = inx ? X.bH * pzx[v] + X.cH * dEyx : 0.f;
                if (o) {
                    hx_jm[v] = ahx[v] - adb[v] * ((Ym.kH * dEzy + vxy) - (idzH * dEyz));
                    hz_jm[v] = ahz[v] - adb[v] * ((X.kH * dEyx + vzx) - (Ym.kH * dExy + vzy));
                }
            }
            if (PZ && zany && o) {
                float oz[V], kh[V], bh[V], chh[V];
                zload(oz, kh, bh, chh, P0[PSI_HXZ], zs3(i, j - 1, 0, ny, sz), p.z.kH, p.z.bH, p.z.cH);
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if (zsv[v] >= 0) {
                        const float pxz = bh[v] * oz[v] + chh[v] * dEyzB[v];
                        hx_jm[v] += adb[v] * ((kh[v] - idzH) * dEyzB[v] + pxz);
                    }
            }
        }

        // ---- Hx, Hy at z = ks-1 (first active lane of the segment), then the
        // z-1 neighbours ----
        float hx_l = 0.f, hy_l = 0.f;
        if (ok && first && km >= 0) {
            const unsigned q0 = r0 + km;
            const float lex = ex0[q0], ley = ey0[q0], lez = ez0[q0];
            const float lezy = yj ? ez0[q0 + sys] : 0.f;
            const float lezx = xi ? ez0[q0 + sxs] : 0.f;
            const float ldb = MAT == 2 ? p.db[q0] : p.db0;
            const float dEzy = lezy - lez, dEyz = ey[0] - ley;
            const float dExz = ex[0] - lex, dEzx = lezx - lez;
            float a = Y.kH * dEzy, b2 = X.kH * dEzx;
            if (PXY) {
                if (Y.s >= 0) a += Y.bH * P0[PSI_HXY][ys3(i, Y.s, km, sy, nz)] + Y.cH * dEzy;
                if (X.s >= 0) b2 += X.bH * P0[PSI_HYX][xs3(X.s, j, km, ny, nz)] + X.cH * dEzx;
            }
            hx_l = hx0[q0] - ldb * (a - idzH * dEyz);
            hy_l = hy0[q0] - ldb * (idzH * dExz - b2);
            if (PZ) {
                const int zs = slab_index(p.z, km);
                if (zs >= 0) {
                    const unsigned qz = zs3(i, j, zs, ny, sz);
                    const float zk = p.z.kH[km] - idzH, zb = p.z.bH[km], zc = p.z.cH[km];
                    hx_l += ldb * (zk * dEyz + (zb * P0[PSI_HXZ][qz] + zc * dEyz));
                    hy_l -= ldb * (zk * dExz + (zb * P0[PSI_HYZ][qz] + zc * dExz));
                }
            }
        }
        float hxm[V], hym[V];
#pragma unroll
        for (int v = 1; v < V; ++v) {
            hxm[v] = hx[v - 1];
            hym[v] = hy[v - 1];
        }
        {
            const float s1 = lane_prev(hx[V - 1]), s2 = lane_prev(hy[V - 1]);
            hxm[0] = first ? hx_l : s1;
            hym[0] = first ? hy_l : s2;
        }

        // ---- E layer at the own cells ----
        float exw[V], eyw[V], ezw[V];
        {
            float dHyzA[V], dHxzA[V];
            float pxy[V], pzy[V], pyx[V], pzx[V];
            const bool iny = PXY && ok && Y.s >= 0, inx = PXY && ok && X.s >= 0;
            const unsigned qy = iny ? ys3(i, Y.s, kb, sy, nz) : 0, qx = inx ? xs3(X.s, j, kb, ny, nz) : 0;
            ld(pxy, P0[PSI_EXY], qy, iny);
            ld(pzy, P0[PSI_EZY], qy, iny);
            ld(pyx, P0[PSI_EYX], qx, inx);
            ld(pzx, P0[PSI_EZX], qx, inx);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int k = kb + v;
                exw[v] = ex[v];
                eyw[v] = ey[v];
                ezw[v] = ez[v];
                const float dHzy = hz[v] - hz_jm[v], dHyz = hy[v] - hym[v];
                const float dHxz = hx[v] - hxm[v], dHzx = hz[v] - hzp[v];
                const float dHyx = hy[v] - hyp[v], dHxy = hx[v] - hx_jm[v];
                dHyzA[v] = dHyz;
                dHxzA[v] = dHxz;
                if (jm && k >= 1) {
                    if (iny) pxy[v] = Y.bE * pxy[v] + Y.cE * dHzy;
                    const float a = Y.kE * dHzy + (iny ? pxy[v] : 0.f), b = idzE * dHyz;
                    exw[v] = (MAT >= 1 ? ca[v] * ex[v] : ex[v]) + cb[v] * (a - b);
                }
                if (im && k >= 1) {
                    if (inx) pyx[v] = X.bE * pyx[v] + X.cE * dHzx;
                    const float a = idzE * dHxz, b = X.kE * dHzx + (inx ? pyx[v] : 0.f);
                    eyw[v] = (MAT >= 1 ? ca[v] * ey[v] : ey[v]) + cb[v] * (a - b);
                }
                if (im && jm) {
                    if (inx) pzx[v] = X.bE * pzx[v] + X.cE * dHyx;
                    if (iny) pzy[v] = Y.bE * pzy[v] + Y.cE * dHxy;
                    const float a = X.kE * dHyx + (inx ? pzx[v] : 0.f), b = Y.kE * dHxy + (iny ? pzy[v] : 0.f);
                    ezw[v] = (MAT >= 1 ? ca[v] * ez[v] : ez[v]) + cb[v] * (a - b);
                }
            }
            if (PZ && zany) {
                // z-slab psi of Ex, Ey; cells the E layer does not update keep
                // their (zero) value
                const unsigned row = zrow;
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if (zsv[v] >= 0) {
                        const int k = kb + v;
                        const float kz = p.z.kE[k], bz = p.z.bE[k], cz = p.z.cE[k];
                        float o3 = zo[2][v], o4 = zo[3][v];
                        if (jm && k >= 1) {
                            o3 = bz * o3 + cz * dHyzA[v];
                            exw[v] -= cb[v] * ((kz - idzE) * dHyzA[v] + o3);
                        }
                        if (im && k >= 1) {
                            o4 = bz * o4 + cz * dHxzA[v];
                            eyw[v] += cb[v] * ((kz - idzE) * dHxzA[v] + o4);
                        }
                        P1[PSI_EXZ][row + zsv[v]] = o3;
                        P1[PSI_EYZ][row + zsv[v]] = o4;
                    }
            }
#pragma unroll
            for (int v = 0; v < V; ++v)
                if (p.src_idx >= 0 && ok && in_src(p.src_box, i, j, kb + v)) {
                    const float sval = step < p.src_len ? p.src_vals[step] : 0.f;
                    if (p.src_comp == FDTD_EX) exw[v] += sval;
                    else if (p.src_comp == FDTD_EY) eyw[v] += sval;
                    else ezw[v] += sval;
                }
            // psi of cells the E layer does not update keep their (zero) value
            if (iny) { stv<V>(P1[PSI_EXY] + qy, pxy); stv<V>(P1[PSI_EZY] + qy, pzy); }
            if (inx) { stv<V>(P1[PSI_EYX] + qx, pyx); stv<V>(P1[PSI_EZX] + qx, pzx); }
        }
        if (ok) {
            stv<V>(p.s1.f[FDTD_EX] + c, exw);
            stv<V>(p.s1.f[FDTD_EY] + c, eyw);
            stv<V>(p.s1.f[FDTD_EZ] + c, ezw);
            stv<V>(p.s1.f[FDTD_HX] + c, hx);
            stv<V>(p.s1.f[FDTD_HY] + c, hy);
            stv<V>(p.s1.f[FDTD_HZ] + c, hz);
        }
        // ---- probes in this plane (grouped by x plane and 4-row band) ----
        if (pt.start != nullptr && T.rec) {
            const int g = i * ((ny + 3) / 4) + jr / 4;
            const int pend = pt.start[g + 1];
            for (int q = pt.start[g]; q < pend; ++q) {
                const int64_t cell = pt.cell[q];
                if (!ok || cell < (int64_t)c || cell >= (int64_t)c + V) continue;
                const int v = (int)(cell - c);
                float val = 0.f;
#pragma unroll
                for (int w = 0; w < V; ++w) {
                    if (w != v) continue;
                    switch (p.probe_comp) {
                        case FDTD_EX: val = exw[w]; break;
                        case FDTD_EY: val = eyw[w]; break;
                        case FDTD_EZ: val = ezw[w]; break;
                        case FDTD_HX: val = hx[w]; break;
                        case FDTD_HY: val = hy[w]; break;
                        default: val = hz[w]; break;
                    }
                }
                p.rec[(int64_t)pt.slot[q] * p.rec_stride + (step - p.rec_base)] = val;
            }
        }
        // carry to the next plane
#pragma unroll
        for (int v = 0; v < V; ++v) {
            eyc[v] = ey_x[v];
            ezc[v] = ez_x[v];
            hyp[v] = hy[v];
            hzp[v] = hz[v];
        }
    }
}

template <int V, int WPB, bool PXY, bool PZ, int MAT>
static void go(const Prob3D &p, const Wave3DLaunch &l, const Tile3 *tiles, const ProbeTiles &pt,
               int64_t step, hipStream_t st) {
    hipLaunchKernelGGL((k3d_march<V, WPB, PXY, PZ, MAT>), dim3((unsigned)l.n), dim3(64 * WPB), 0, st, p,
                       tiles + l.off, pt, step);
}

template <int V, int WPB, bool PXY, bool PZ>
static void go_m(const Prob3D &p, const Wave3DLaunch &l, const Tile3 *tiles, const ProbeTiles &pt,
                 int64_t step, hipStream_t st) {
    const int mat = p.db ? 2 : (p.ca ? 1 : 0);
    if (mat == 0) go<V, WPB, PXY, PZ, 0>(p, l, tiles, pt, step, st);
    else if (mat == 1) go<V, WPB, PXY, PZ, 1>(p, l, tiles, pt, step, st);
    else go<V, WPB, PXY, PZ, 2>(p, l, tiles, pt, step, st);
}

// interior launches: 8-row workgroups; x/y-slab launches: 4-row ones
template <int V>
static void go_v(const Prob3D &p, const Wave3DLaunch &l, const Tile3 *tiles, const ProbeTiles &pt,
                 int64_t step, hipStream_t st) {
    if (l.pxy) {
        if (l.pz) go_m<V, 4, true, true>(p, l, tiles, pt, step, st);
        else go_m<V, 4, true, false>(p, l, tiles, pt, step, st);
    } else {
        if (l.pz) go_m<V, 8, false, true>(p, l, tiles, pt, step, st);
        else go_m<V, 8, false, false>(p, l, tiles, pt, step, st);
    }
}

hipError_t launch_3d_wave(const Prob3D &p, const Wave3DPlan &pl, const Tile3 *tiles, const ProbeTiles &pt,
                          int64_t step, hipStream_t st, hipEvent_t *ev) {
    int q = 0;
    for (const Wave3DLaunch &l : pl.l) {
        if (ev) {
            const hipError_t e = hipEventRecord(ev[q++], st);
            if (e != hipSuccess) return e;
        }
        if (l.wpb != (l.pxy ? 4 : 8)) return hipErrorInvalidValue;
        if (l.V == 4) go_v<4>(p, l, tiles, pt, step, st);
        else if (l.V == 2) go_v<2>(p, l, tiles, pt, step, st);
        else if (l.V == 1) go_v<1>(p, l, tiles, pt, step, st);
        else return hipErrorInvalidValue;
    }
    if (ev) {
        const hipError_t e = hipEventRecord(ev[q], st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace gem
