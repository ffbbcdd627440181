// Two leapfrog steps per pass over HBM (temporal blocking) for the 3D grid:
// state n is read once, state n+2 written once, state n+1 lives in
// registers and LDS only (its x/y-slab psi excepted, see below).
//
// A workgroup holds R+2 y rows (its R rows plus one halo row above and one
// below) of full z length (RZ wavefronts of 64 lanes x V cells per row) and
// marches through the x planes of its tile.  At plane i it computes step 1
// (H^{n+1/2}, E^{n+1}) of all its rows at plane i, then step 2 (H^{n+3/2},
// E^{n+2}) of its own rows at plane i-1, which needs step 1 at planes i-1
// and i only:
//   x: step-1 values of plane i-1 are carried in registers; the tile starts
//      one plane early and recomputes H^{n+1/2} (y, z) of the plane before;
//   y: rows exchange through LDS; the halo rows give step 1 of the rows
//      next to the band (the upper one recomputes H^{n+1/2} of the row above
//      it from state n, the lower one loads E^n of the row below);
//   z: the lane shuffle and, between wavefronts of a row, LDS seam values;
//      the row is whole, so no z halo.
// Step-1 values of the halo rows and planes are recomputed by every tile
// that needs them, identically, so tiles stay independent (no grid barrier).
// z-slab CPML: correction of the slab lanes as in the single-step kernel;
// their step-1 psi values wait in LDS (indexed by slab cell) until step 2.
// x/y-slab CPML (instances with PXY, for the tiles whose dependency cone,
// planes i0-2 .. i1 and rows j0-2 .. j0+R, touches an x or y slab; the
// others run without that code): the plane's and the row's profiles are
// wave-uniform scalars; the step-1 psi of a slab cell goes to the psi
// arrays of a third state set (the same thread reads it back at the next
// plane; a halo row's value, written by two tiles, is the same in both).
// The tiles near one slab kind run a kernel with a code path per kind
// (SL 4: each without the other kind's psi code, chosen per tile); those
// near both kinds an instance with all of it (SL 3).
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "devutil.hpp"
#include "k3dcell.hpp"

namespace gem {

// Step-2 H in LDS buffers of its own, so that no barrier has to wait for
// the step-1 reads of LHx, LHz before it is written: 12-wavefront instances
// without x/y-slab code or a Db map (the others would spill, or exceed the
// LDS, with 2 x NT x V floats more).
constexpr bool two_sb(bool pxy, int mat, int waves) { return !pxy && mat != 2 && waves == 12; }

// The workgroup's LDS arrays (declared once per kernel, shared by the code
// paths of a kernel that holds two).  z-slab data, ZW entries per row: entry e holds
// cell k = e below LO4 (the low slab's size rounded up to a multiple of 4)
// and k = HB4 + e - LO4 from LO4 on (HB4: start of the high slab rounded
// down), so a lane's V cells are V aligned consecutive entries; entries of
// cells outside the slabs are padding (profile 0, psi 0: the correction is
// then exactly zero).
//   ZT: profile (kH - idzH, bH, cH, kE - idzE, bE, cE)
//   ZP: state-n psi (Hx-z, Hy-z, Ex-z, Ey-z) of the current plane, rows
//       j0-2 .. j0+R, copied from memory with the plane's fields
//   Zs: step-1 psi of the last two planes (by plane parity) for step 2
//   ZQ: step-2 psi of the own rows, written to memory coalesced after the
//       next barrier
template <int V, int RZ, int R, bool PZ, bool SB>
struct TwoLds {
    static constexpr int NR = R + 2, NT = 64 * RZ * NR, ZW = kTwoZMax + 8, NZR = NR + 1;
    float (&LEx)[NT * V], (&LEz)[NT * V], (&LHx)[NT * V], (&LHz)[NT * V], (&L1x)[NT * V], (&L1z)[NT * V];
    float (&LH2x)[SB ? NT * V : 1], (&LH2z)[SB ? NT * V : 1];
    float (&Se0)[NR][RZ][2], (&Sh1)[NR][RZ][2], (&Se1)[NR][RZ][2], (&Sh2)[NR][RZ][2];
    float (&ZT)[PZ ? 6 : 1][PZ ? ZW : 4];
    float (&ZP)[PZ ? 4 : 1][PZ ? NZR * ZW : 4];
    float (&Zs)[PZ ? 2 : 1][PZ ? NR : 1][PZ ? 4 : 1][PZ ? ZW : 4];
    float (&ZQ)[PZ ? 4 : 1][PZ ? R * ZW : 4];
};

// One tile (T, at index tix of the launch's list) of the two-step pass.
// SL: slab kinds of the instance's tiles (x/y-slab code): bit 0 x, bit 1 y;
// the ψ code of a kind absent is left out.
template <int V, int RZ, int R, bool PZ, bool PXY, int MAT, bool REC, int SL, class Lds>
__device__ __forceinline__ void two_tile(const Prob3D &p, const TileTB &T, int tix, const ProbeTiles &pt,
                                         int64_t step, const State3D &mid, Lds &L) {
    constexpr int NR = R + 2;            // rows held: halo, R own, halo
    constexpr int NT = 64 * RZ * NR;     // threads
    constexpr int SEG = 64 * V;          // z cells per wavefront
    constexpr int ROW = RZ * SEG;        // LDS floats per row
    constexpr bool SX = PXY && (SL & 1) != 0, SY = PXY && (SL & 2) != 0;
    // whether this tile records probes (wave-uniform)
    const bool tprobe = REC && pt.start != nullptr && (pt.tile_any == nullptr || pt.tile_any[tix] != 0);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int seg = w % RZ, rr = w / RZ;
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int j = T.j0 - 1 + rr;
    const bool top = rr == 0, bot = rr == T.nrows + 1;
    const bool own = rr >= 1 && rr <= T.nrows;
    const bool rok = rr <= T.nrows + 1 && j >= 0 && j < ny;
    const int kb = seg * SEG + lane * V;
    const bool ok = rok && kb < nz;  // nz % V == 0
    const int segend = min((seg + 1) * SEG, nz);
    const bool last = kb + V == segend, seamnext = segend < nz;
    const bool yj = j + 1 < ny, jm = j >= 1;
    const unsigned sxs = (unsigned)ny * nz, sys = nz;
    const int jr = rok ? j : 0;
    const int sz = p.z.lo + p.z.hi;
    const float *ex0 = p.s0.f[FDTD_EX], *ey0 = p.s0.f[FDTD_EY], *ez0 = p.s0.f[FDTD_EZ];
    const float *hx0 = p.s0.f[FDTD_HX], *hy0 = p.s0.f[FDTD_HY], *hz0 = p.s0.f[FDTD_HZ];
    float *const *P0 = p.s0.psi;
    float *const *P1 = p.s1.psi;
    float *const *PM = mid.psi;  // x/y-slab psi of state n+1 (PXY)
    const int sy = p.y.lo + p.y.hi;
    const int tq = (int)threadIdx.x * V;
    // x and y profiles: without x/y-slab code the interior ones (no slab in
    // the cone), else those of the plane and the row
    const float ikx = p.x.kH[p.x.lo], iky = p.y.kH[p.y.lo], jkx = p.x.kE[p.x.lo], jky = p.y.kE[p.y.lo];
    const float idzH = p.z.kH[p.z.lo], idzE = p.z.kE[p.z.lo];
    auto prof = [&](const AxisDev &a, int q, float kh, float ke) {
        if constexpr (PXY) return axp<true>(a, q);
        else return AxP{kh, ke, 0.f, 0.f, 0.f, 0.f, -1};
    };
    const AxP Y = prof(p.y, jr, iky, jky);                             // row j

    constexpr bool SB = two_sb(PXY, MAT, NR * RZ);
    auto &LEx = L.LEx, &LEz = L.LEz, &LHx = L.LHx, &LHz = L.LHz, &L1x = L.L1x, &L1z = L.L1z;
    auto &Se0 = L.Se0, &Sh1 = L.Sh1, &Se1 = L.Se1, &Sh2 = L.Sh2;
    auto &ZT = L.ZT;
    auto &ZP = L.ZP;
    auto &Zs = L.Zs;
    auto &ZQ = L.ZQ;
    float *const H2x = SB ? L.LH2x : L.LHx, *const H2z = SB ? L.LH2z : L.LHz;
    constexpr int ZW = kTwoZMax + 8;
    constexpr int NZR = NR + 1;
    const int zlo = p.z.lo, zhi = p.z.hi;
    const int LO4 = (zlo + 3) & ~3, HB4 = (nz - zhi) & ~3;
    const bool zany = PZ && ok && (kb < LO4 || kb >= HB4);
    const int zl = PZ ? (kb < LO4 ? kb : LO4 + kb - HB4) : 0;
    // entry e: its cell's slab index s (the psi arrays' z index); true if the
    // cell lies in a slab
    auto zent = [&](int e, int &zs) {
        if (e < LO4) {
            zs = e;
            return e < zlo;
        }
        const int k = HB4 + e - LO4;
        zs = zlo + (k - (nz - zhi));
        return k >= nz - zhi && k < nz;
    };

    auto zero = [](float (&a)[V]) {
#pragma unroll
        for (int v = 0; v < V; ++v) a[v] = 0.f;
    };
    auto ld = [&](float (&a)[V], const float *base, unsigned off, bool cond) {
        if (cond) ldv<V>(a, base + off);
        else zero(a);
    };
    auto prv = [&](const float (&x)[V], int q, float seam) {
        if (q > 0) return x[q - 1];
        const float s = lane_prev(x[V - 1]);
        return lane == 0 ? seam : s;
    };
    // H from E: own, +x, +y, +z seam; the z differences are kept for the
    // slab correction.  Xa, Ya: profiles of the cells' plane and row.  With
    // x/y-slab code, q holds the psi of the slabs the cells lie in (old in,
    // new out): q[0] Hx-y, q[1] Hz-y (y slab: iny), q[2] Hy-x, q[3] Hz-x
    // (x slab: inx).
    auto hstep = [&](float (&hx)[V], float (&hy)[V], float (&hz)[V], const float (&db)[V], const float (&ex)[V],
                     const float (&ey)[V], const float (&ez)[V], const float (&eyx)[V], const float (&ezx)[V],
                     const float (&exy)[V], const float (&ezy)[V], float exs, float eys, float (&dyz)[V],
                     float (&dxz)[V], const AxP &Xa, const AxP &Ya, bool inx, bool iny, float (&q)[4][V]) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const float dEzy = ezy[v] - ez[v];
            const float dEyz = znext<V>(ey, v, eys, last) - ey[v];
            const float dExz = znext<V>(ex, v, exs, last) - ex[v];
            const float dEzx = ezx[v] - ez[v], dEyx = eyx[v] - ey[v], dExy = exy[v] - ex[v];
            dyz[v] = dEyz;
            dxz[v] = dExz;
            float ty = Ya.kH * dEzy, tzy = Ya.kH * dExy, tx = Xa.kH * dEzx, tzx = Xa.kH * dEyx;
            if (SY && iny) {
                q[0][v] = Ya.bH * q[0][v] + Ya.cH * dEzy;
                q[1][v] = Ya.bH * q[1][v] + Ya.cH * dExy;
                ty += q[0][v];
                tzy += q[1][v];
            }
            if (SX && inx) {
                q[2][v] = Xa.bH * q[2][v] + Xa.cH * dEzx;
                q[3][v] = Xa.bH * q[3][v] + Xa.cH * dEyx;
                tx += q[2][v];
                tzx += q[3][v];
            }
            hx[v] = hx[v] - db[v] * (ty - (idzH * dEyz));
            hy[v] = hy[v] - db[v] * ((idzH * dExz) - tx);
            hz[v] = hz[v] - db[v] * (tzx - tzy);
        }
    };
    // z-slab correction of H (psi in o1 = Hx-z, o2 = Hy-z: old in, new out)
    auto hfix = [&](float (&hx)[V], float (&hy)[V], const float (&db)[V], const float (&dyz)[V],
                    const float (&dxz)[V], float (&o1)[V], float (&o2)[V], bool fx, bool fy) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const float kh = ZT[0][zl + v], bh = ZT[PZ ? 1 : 0][zl + v], ch = ZT[PZ ? 2 : 0][zl + v];
            o1[v] = bh * o1[v] + ch * dyz[v];
            o2[v] = bh * o2[v] + ch * dxz[v];
            if (fx) hx[v] += db[v] * (kh * dyz[v] + o1[v]);
            if (fy) hy[v] -= db[v] * (kh * dxz[v] + o2[v]);
        }
    };
    // E from H: own, -x, -y, -z seam (ex/ey/ez old in, new out).  With
    // x/y-slab code, q: q[0] Ex-y, q[1] Ez-y (y slab), q[2] Ey-x, q[3] Ez-x
    // (x slab); the psi of a cell the E layer does not update stays.
    auto estep = [&](float (&ex)[V], float (&ey)[V], float (&ez)[V], const float (&ca)[V], const float (&cb)[V],
                     const float (&hx)[V], const float (&hy)[V], const float (&hz)[V], const float (&hyp)[V],
                     const float (&hzp)[V], const float (&hxj)[V], const float (&hzj)[V], float hxs, float hys,
                     bool im, float (&dyz)[V], float (&dxz)[V], const AxP &Xa, const AxP &Ya, bool inx, bool iny,
                     float (&q)[4][V]) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            dyz[v] = hy[v] - prv(hy, v, hys);
            dxz[v] = hx[v] - prv(hx, v, hxs);
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int k = kb + v;
            const float dHzy = hz[v] - hzj[v], dHzx = hz[v] - hzp[v];
            const float dHyx = hy[v] - hyp[v], dHxy = hx[v] - hxj[v];
            const bool ux = jm && k >= 1, uy = im && k >= 1, uz = im && jm;
            float ty = Ya.kE * dHzy, tx = Xa.kE * dHzx, tzx = Xa.kE * dHyx, tzy = Ya.kE * dHxy;
            if (SY && iny) {
                if (ux) q[0][v] = Ya.bE * q[0][v] + Ya.cE * dHzy;
                if (uz) q[1][v] = Ya.bE * q[1][v] + Ya.cE * dHxy;
                ty += q[0][v];
                tzy += q[1][v];
            }
            if (SX && inx) {
                if (uy) q[2][v] = Xa.bE * q[2][v] + Xa.cE * dHzx;
                if (uz) q[3][v] = Xa.bE * q[3][v] + Xa.cE * dHyx;
                tx += q[2][v];
                tzx += q[3][v];
            }
            if (ux) ex[v] = (MAT >= 1 ? ca[v] * ex[v] : ex[v]) + cb[v] * (ty - (idzE * dyz[v]));
            if (uy) ey[v] = (MAT >= 1 ? ca[v] * ey[v] : ey[v]) + cb[v] * ((idzE * dxz[v]) - tx);
            if (uz) ez[v] = (MAT >= 1 ? ca[v] * ez[v] : ez[v]) + cb[v] * (tzx - tzy);
        }
    };
    // x/y-slab psi of the thread's cells: q[0], q[1] from the y-slab arrays
    // a, b at qy (if iny), q[2], q[3] from the x-slab arrays c, d at qx (if
    // inx), else zero; and the reverse
    auto qload = [&](float (&q)[4][V], float *const *S, int a, int b, int c, int d, unsigned qy, bool iny,
                     unsigned qx, bool inx) {
        ld(q[0], S[a], qy, SY && iny);
        ld(q[1], S[b], qy, SY && iny);
        ld(q[2], S[c], qx, SX && inx);
        ld(q[3], S[d], qx, SX && inx);
    };
    auto qstore = [&](const float (&q)[4][V], float *const *S, int a, int b, int c, int d, unsigned qy, bool iny,
                      unsigned qx, bool inx) {
        if (SY && iny) {
            stv<V>(S[a] + qy, q[0]);
            stv<V>(S[b] + qy, q[1]);
        }
        if (SX && inx) {
            stv<V>(S[c] + qx, q[2]);
            stv<V>(S[d] + qx, q[3]);
        }
    };
    // z-slab correction of E (o3 = Ex-z, o4 = Ey-z); cells not updated keep psi
    auto efix = [&](float (&ex)[V], float (&ey)[V], const float (&cb)[V], const float (&dyz)[V],
                    const float (&dxz)[V], float (&o3)[V], float (&o4)[V], bool im) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const float ke = ZT[PZ ? 3 : 0][zl + v], be = ZT[PZ ? 4 : 0][zl + v], ce = ZT[PZ ? 5 : 0][zl + v];
            const bool kk = kb + v >= 1;
            if (jm && kk) {
                o3[v] = be * o3[v] + ce * dyz[v];
                ex[v] -= cb[v] * (ke * dyz[v] + o3[v]);
            }
            if (im && kk) {
                o4[v] = be * o4[v] + ce * dxz[v];
                ey[v] += cb[v] * (ke * dxz[v] + o4[v]);
            }
        }
    };
    // psi of the thread's cells from the LDS copy (component cc, row index
    // r = j - (j0 - 2))
    auto zlds = [&](float (&o)[V], int cc, int r) { ldv<V>(o, &ZP[PZ ? cc : 0][PZ ? r * ZW + zl : 0]); };
    // from memory (tile start only): padding cells read as 0
    auto zload = [&](float (&o)[V], const float *a, unsigned row) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int q = slab_index(p.z, kb + v);
            o[v] = q >= 0 ? a[row + q] : 0.f;
        }
    };
    // step-1 stash and step-2 output of the thread's cells
    auto zstash_w = [&](int par, int cc, const float (&o)[V]) { stv<V>(&Zs[PZ ? par : 0][PZ ? rr : 0][PZ ? cc : 0][zl], o); };
    auto zstash_r = [&](float (&o)[V], int par, int cc) { ldv<V>(o, &Zs[PZ ? par : 0][PZ ? rr : 0][PZ ? cc : 0][zl]); };
    auto zout = [&](int cc, const float (&o)[V]) { stv<V>(&ZQ[PZ ? cc : 0][PZ ? (rr - 1) * ZW + zl : 0], o); };
    // coalesced copy of the step-2 psi of plane ib (own rows) to memory
    auto zflush = [&](int ib) {
        for (int q = (int)threadIdx.x; q < R * ZW; q += NT) {
            const int r = q / ZW, e = q - r * ZW;
            int zs;
            if (zent(e, zs) && r < T.nrows) {
                const unsigned g = zs3(ib, T.j0 + r, zs, ny, sz);
                P1[PSI_HXZ][g] = ZQ[0][q];
                P1[PSI_HYZ][g] = ZQ[PZ ? 1 : 0][q];
                P1[PSI_EXZ][g] = ZQ[PZ ? 2 : 0][q];
                P1[PSI_EYZ][g] = ZQ[PZ ? 3 : 0][q];
            }
        }
    };
    // The element is picked by selects, never by an index computed at run
    // time: a computed index into a register array moves the array to
    // scratch memory for the whole kernel.
    auto add_source = [&](int i, int64_t n, float (&ex)[V], float (&ey)[V], float (&ez)[V]) {
        const int *b = p.src_box;
        if (p.src_idx < 0 || !ok || (unsigned)(i - b[0]) >= (unsigned)(b[1] - b[0]) ||
            (unsigned)(j - b[2]) >= (unsigned)(b[3] - b[2]))
            return;
        const float sval = n < p.src_len ? p.src_vals[n] : 0.f;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const bool at = (unsigned)(kb + v - b[4]) < (unsigned)(b[5] - b[4]);
            ex[v] = (at && p.src_comp == FDTD_EX) ? ex[v] + sval : ex[v];
            ey[v] = (at && p.src_comp == FDTD_EY) ? ey[v] + sval : ey[v];
            ez[v] = (at && p.src_comp == FDTD_EZ) ? ez[v] + sval : ez[v];
        }
    };
    auto record = [&](int i, unsigned c, int64_t n, const float (&ex)[V], const float (&ey)[V], const float (&ez)[V],
                      const float (&hx)[V], const float (&hy)[V], const float (&hz)[V]) {
        if (!REC || !tprobe || !ok) return;
        const int g = i * ((ny + 3) / 4) + jr / 4;
        const int pend = pt.start[g + 1];
        for (int q = pt.start[g]; q < pend; ++q) {
            const int64_t cell = pt.cell[q];
            if (cell < (int64_t)c || cell >= (int64_t)c + V) continue;
            const int v = (int)(cell - c);
            const int pc = p.probe_comp;
            float val = 0.f;
#pragma unroll
            for (int u = 0; u < V; ++u) {
                const float x = pc == FDTD_EX ? ex[u] : pc == FDTD_EY ? ey[u] : pc == FDTD_EZ ? ez[u]
                              : pc == FDTD_HX ? hx[u] : pc == FDTD_HY ? hy[u] : hz[u];
                val = u == v ? x : val;
            }
            p.rec[(int64_t)pt.slot[q] * p.rec_stride + (n - p.rec_base)] = val;
        }
    };
    auto coef = [&](float (&cb)[V], float (&ca)[V], float (&db)[V], unsigned c, bool cond) {
        ld(cb, p.cb, c, cond);
#pragma unroll
        for (int v = 0; v < V; ++v) { ca[v] = 1.f; db[v] = p.db0; }
        if (MAT >= 1 && cond) ldv<V>(ca, p.ca + c);
        if (MAT == 2 && cond) ldv<V>(db, p.db + c);
    };

    const int ia = T.i0 > 0 ? T.i0 - 1 : 0;
    if (PZ) {  // profile table; psi copy zeroed (its padding stays zero)
        for (int q = (int)threadIdx.x; q < 6 * ZW; q += NT) {
            const int c = q / ZW, e = q - c * ZW;
            int zs;
            const bool real = zent(e, zs);
            const int k = e < LO4 ? e : HB4 + e - LO4;
            float v = 0.f;
            if (real) {
                v = c == 0 ? p.z.kH[k] - idzH : c == 1 ? p.z.bH[k] : c == 2 ? p.z.cH[k]
                  : c == 3 ? p.z.kE[k] - idzE : c == 4 ? p.z.bE[k] : p.z.cE[k];
            }
            ZT[PZ ? c : 0][e] = v;
        }
        for (int q = (int)threadIdx.x; q < 4 * NZR * ZW; q += NT) (&ZP[0][0])[q] = 0.f;
        __syncthreads();
    }
    // carried between planes
    float eyc[V], ezc[V];             // E^n at plane i
    float hx1p[V], hy1p[V], hz1p[V];  // H^{n+1/2} at plane i-1
    float ex1p[V], ey1p[V], ez1p[V];  // E^{n+1} at plane i-1
    float hy2p[V], hz2p[V];           // H^{n+3/2} at plane i-2
    float cbp[V], cap[V], dbp[V];     // coefficients at plane i-1
    zero(hx1p); zero(hy1p); zero(hz1p); zero(ex1p); zero(ey1p); zero(ez1p); zero(hy2p); zero(hz2p);
#pragma unroll
    for (int v = 0; v < V; ++v) { cbp[v] = 0.f; cap[v] = 1.f; dbp[v] = p.db0; }
    {
        const unsigned c = ((unsigned)ia * ny + jr) * nz + kb;
        ld(eyc, ey0, c, ok);
        ld(ezc, ez0, c, ok);
        if (ia >= 1) {  // H^{n+1/2} (y, z) at plane ia-1 from state n
            const unsigned q0 = c - sxs;
            float aex[V], aey[V], aez[V], aexy[V], ahx[V], ahy[V], ahz[V], ab[V], aa[V], adb[V], dyz[V], dxz[V];
            ld(aex, ex0, q0, ok);
            ld(aey, ey0, q0, ok);
            ld(aez, ez0, q0, ok);
            ld(aexy, ex0, q0 + sys, ok && yj);
            zero(ahx);
            ld(ahy, hy0, q0, ok);
            ld(ahz, hz0, q0, ok);
            coef(ab, aa, adb, q0, ok);
            const unsigned rq = ((unsigned)(ia - 1) * ny + jr) * nz;
            const bool sn = ok && last && seamnext;
            const float exs = sn ? ex0[rq + segend] : 0.f, eys = sn ? ey0[rq + segend] : 0.f;
            float zz[V];
            zero(zz);
            const AxP Xq = prof(p.x, ia - 1, ikx, jkx);
            float qa[4][V];  // Hx-y unused (Hx is not needed)
            const bool inx = PXY && ok && Xq.s >= 0, iny = PXY && ok && Y.s >= 0;
            if (PXY)
                qload(qa, P0, PSI_HXY, PSI_HZY, PSI_HYX, PSI_HZX, iny ? ys3(ia - 1, Y.s, kb, sy, nz) : 0, iny,
                      inx ? xs3(Xq.s, j, kb, ny, nz) : 0, inx);
            hstep(ahx, ahy, ahz, adb, aex, aey, aez, eyc, ezc, aexy, zz, exs, eys, dyz, dxz, Xq, Y, inx, iny, qa);
            if (PZ && zany) {
                float o1[V], o2[V];
                zload(o1, P0[PSI_HXZ], zs3(ia - 1, j, 0, ny, sz));
                zload(o2, P0[PSI_HYZ], zs3(ia - 1, j, 0, ny, sz));
                hfix(ahx, ahy, adb, dyz, dxz, o1, o2, false, true);
            }
#pragma unroll
            for (int v = 0; v < V; ++v) { hy1p[v] = ahy[v]; hz1p[v] = ahz[v]; }
        }
    }
    float ex1y[V], ez1y[V];  // E^{n+1} at (i-1, j+1)
    float e1s[2] = {0.f, 0.f};
    zero(ex1y);
    zero(ez1y);

    const int iend = min(T.i1, nx);
    // Without x/y-slab code, Ex, Hx, Hy, Hz of the next plane are loaded
    // before the current plane's second step, so that their latency overlaps
    // it (the waves of a workgroup would otherwise all wait for them at the
    // plane's first barrier).  The instances with x/y-slab code or a Ca
    // map have no registers to spare for them (they would spill).
    constexpr bool PF = !PXY && MAT == 0;
    float pf_ex[V], pf_hx[V], pf_hy[V], pf_hz[V];
    auto prefetch = [&](int in) {
        const bool lan = in < nx && in <= iend && ok;
        const unsigned cn = ((unsigned)(lan ? in : 0) * ny + jr) * nz + kb;
        ld(pf_ex, ex0, cn, lan);
        ld(pf_hx, hx0, cn, lan);
        ld(pf_hy, hy0, cn, lan);
        ld(pf_hz, hz0, cn, lan);
    };
    if (PF) prefetch(ia);
    for (int i = ia; i <= iend; ++i) {
        const bool pa = i < nx;
        const bool xi = i + 1 < nx, im = i >= 1;
        const unsigned r0 = ((unsigned)(pa ? i : 0) * ny + jr) * nz, c = r0 + kb;
        const bool la = pa && ok;
        const AxP X = prof(p.x, pa ? i : 0, ikx, jkx);
        const bool inx1 = PXY && la && X.s >= 0, iny1 = PXY && la && Y.s >= 0;
        const unsigned qx1 = inx1 ? xs3(X.s, j, kb, ny, nz) : 0, qy1 = iny1 ? ys3(i, Y.s, kb, sy, nz) : 0;
        // ---- state-n z psi of plane i (rows j0-2 .. j0+R): issued now,
        //      written to LDS before the first barrier ----
        constexpr int NZQ = NZR * ZW;  // entries per component
        constexpr int NZL = PZ ? (NZQ + NT - 1) / NT : 1;
        float zpre[4][NZL];
        bool zin[NZL];
        if (PZ) {
#pragma unroll
            for (int u = 0; u < NZL; ++u) {
                const int q = (int)threadIdx.x + u * NT;
                const int row = q / ZW, e = q - row * ZW;
                const int jj = T.j0 - 2 + row;
                int zs = 0;
                zin[u] = q < NZQ && zent(e, zs) && jj >= 0 && jj < ny;
                const unsigned g = zs3(pa ? i : 0, zin[u] ? jj : 0, zin[u] ? zs : 0, ny, sz);
                const bool in = zin[u] && pa;
                zpre[0][u] = in ? P0[PSI_HXZ][g] : 0.f;
                zpre[1][u] = in ? P0[PSI_HYZ][g] : 0.f;
                zpre[2][u] = in ? P0[PSI_EXZ][g] : 0.f;
                zpre[3][u] = in ? P0[PSI_EYZ][g] : 0.f;
            }
        }
        // ---- E^{n+1} at plane i-1 of the row below and the z seam ----
        if (i > ia && rr <= T.nrows) {
            ldv<V>(ex1y, &L1x[tq + ROW]);
            ldv<V>(ez1y, &L1z[tq + ROW]);
            if (seg + 1 < RZ) {
                e1s[0] = Se1[rr][seg + 1][0];
                e1s[1] = Se1[rr][seg + 1][1];
            }
        }
        // ---- step 1 at plane i ----
        float ex[V], ey[V], ez[V], eyx[V], ezx[V], exy[V], ezy[V], hx[V], hy[V], hz[V], cb[V], ca[V], db[V];
#pragma unroll
        for (int v = 0; v < V; ++v) { ey[v] = eyc[v]; ez[v] = ezc[v]; }
        if (PF) {
#pragma unroll
            for (int v = 0; v < V; ++v) { ex[v] = pf_ex[v]; hx[v] = pf_hx[v]; hy[v] = pf_hy[v]; hz[v] = pf_hz[v]; }
        } else {
            ld(ex, ex0, c, la);
        }
        ld(eyx, ey0, c + sxs, la && xi);
        ld(ezx, ez0, c + sxs, la && xi);
        ld(exy, ex0, c + sys, la && yj && bot);
        ld(ezy, ez0, c + sys, la && yj && bot);
        if (!PF) {
            ld(hx, hx0, c, la);
            ld(hy, hy0, c, la);
            ld(hz, hz0, c, la);
        }
        coef(cb, ca, db, c, la);
        // x/y-slab psi of H at (i, j), state n in, n+1 out: issued with the
        // field loads (those of E are issued right before use: registers)
        float q1[4][V];
        if (PXY) qload(q1, P0, PSI_HXY, PSI_HZY, PSI_HYX, PSI_HZX, qy1, iny1, qx1, inx1);
        stv<V>(&LEx[tq], ex);
        stv<V>(&LEz[tq], ez);
        if (lane == 0) { Se0[rr][seg][0] = ex[0]; Se0[rr][seg][1] = ey[0]; }
        if (PZ) {
#pragma unroll
            for (int u = 0; u < NZL; ++u)
                if (zin[u]) {
#pragma unroll
                    for (int cc = 0; cc < 4; ++cc) ZP[PZ ? cc : 0][(int)threadIdx.x + u * NT] = zpre[cc][u];
                }
        }
        __syncthreads();
        // step-2 psi of plane i-2 (written to LDS last iteration) to memory
        if (PZ && i - 2 >= T.i0) zflush(i - 2);
        if (!bot && la && yj) {
            ldv<V>(exy, &LEx[tq + ROW]);
            ldv<V>(ezy, &LEz[tq + ROW]);
        }
        const bool sn = last && seamnext;
        const float exs0 = sn ? Se0[rr][seg + (seg + 1 < RZ)][0] : 0.f;
        const float eys0 = sn ? Se0[rr][seg + (seg + 1 < RZ)][1] : 0.f;
        float dyz[V], dxz[V];
        hstep(hx, hy, hz, db, ex, ey, ez, eyx, ezx, exy, ezy, exs0, eys0, dyz, dxz, X, Y, inx1, iny1, q1);
        // step 2 reads them at plane i (rows up to the last own one)
        if (PXY && rr <= T.nrows && i < iend) qstore(q1, PM, PSI_HXY, PSI_HZY, PSI_HYX, PSI_HZX, qy1, iny1, qx1, inx1);
        if (PZ && zany && la) {  // z-slab psi of step 1: state n in, n+1 to the stash
            float o1[V], o2[V];
            zlds(o1, 0, rr + 1);
            zlds(o2, 1, rr + 1);
            hfix(hx, hy, db, dyz, dxz, o1, o2, true, true);
            zstash_w(i & 1, 0, o1);
            zstash_w(i & 1, 1, o2);
        }
        stv<V>(&LHx[tq], hx);
        stv<V>(&LHz[tq], hz);
        if (lane == 63) { Sh1[rr][seg][0] = hx[V - 1]; Sh1[rr][seg][1] = hy[V - 1]; }
        __syncthreads();
        float hxj[V], hzj[V];
        zero(hxj);
        zero(hzj);
        if (!top) {
            if (la && jm) {
                ldv<V>(hxj, &LHx[tq - ROW]);
                ldv<V>(hzj, &LHz[tq - ROW]);
            }
        } else if (pa && rok && jm) {  // H^{n+1/2} (x, z) at (i, j-1) from state n (wave-uniform)
            const unsigned q0 = c - sys;
            float aex[V], aey[V], aez[V], aeyx[V], ahx[V], ahy[V], ahz[V], ab[V], aa[V], adb[V], zz[V], d1[V], d2[V];
            ld(aex, ex0, q0, ok);
            ld(aey, ey0, q0, ok);
            ld(aez, ez0, q0, ok);
            ld(aeyx, ey0, q0 + sxs, ok && xi);
            ld(ahx, hx0, q0, ok);
            zero(ahy);
            ld(ahz, hz0, q0, ok);
            coef(ab, aa, adb, q0, ok);
            const bool snj = ok && last && seamnext;
            const float eys = snj ? ey0[r0 - sys + segend] : 0.f, exs = snj ? ex0[r0 - sys + segend] : 0.f;
            zero(zz);
            float qa[4][V];  // Hy-x unused (Hy is not needed)
            const AxP Ym = prof(p.y, j - 1, iky, jky);
            const bool inx = PXY && ok && X.s >= 0, iny = PXY && ok && Ym.s >= 0;
            if (PXY)
                qload(qa, P0, PSI_HXY, PSI_HZY, PSI_HYX, PSI_HZX, iny ? ys3(i, Ym.s, kb, sy, nz) : 0, iny,
                      inx ? xs3(X.s, j - 1, kb, ny, nz) : 0, inx);
            hstep(ahx, ahy, ahz, adb, aex, aey, aez, aeyx, zz, ex, ez, exs, eys, d1, d2, X, Ym, inx, iny, qa);
            if (PZ && zany) {
                float q1[V], q2[V];
                zlds(q1, 0, rr);
                zero(q2);
                hfix(ahx, ahy, adb, d1, d2, q1, q2, true, false);
            }
#pragma unroll
            for (int v = 0; v < V; ++v) { hxj[v] = ahx[v]; hzj[v] = ahz[v]; }
        }
        const float hxs1 = (lane == 0 && seg > 0) ? Sh1[rr][seg > 0 ? seg - 1 : 0][0] : 0.f;
        const float hys1 = (lane == 0 && seg > 0) ? Sh1[rr][seg > 0 ? seg - 1 : 0][1] : 0.f;
        float ex1[V], ey1[V], ez1[V];
#pragma unroll
        for (int v = 0; v < V; ++v) { ex1[v] = ex[v]; ey1[v] = ey[v]; ez1[v] = ez[v]; }
        float e1q[4][V];  // x/y-slab psi of E at (i, j): state n in, n+1 out
        if (PXY) qload(e1q, P0, PSI_EXY, PSI_EZY, PSI_EYX, PSI_EZX, qy1, iny1, qx1, inx1);
        estep(ex1, ey1, ez1, ca, cb, hx, hy, hz, hy1p, hz1p, hxj, hzj, hxs1, hys1, im, dyz, dxz, X, Y, inx1, iny1, e1q);
        if (PXY && own && i >= T.i0 && i < iend)  // step 2 of the own rows reads them at plane i
            qstore(e1q, PM, PSI_EXY, PSI_EZY, PSI_EYX, PSI_EZX, qy1, iny1, qx1, inx1);
        if (PZ && zany && la) {
            float o3[V], o4[V];
            zlds(o3, 2, rr + 1);
            zlds(o4, 3, rr + 1);
            efix(ex1, ey1, cb, dyz, dxz, o3, o4, im);
            zstash_w(i & 1, 2, o3);
            zstash_w(i & 1, 3, o4);
        }
        add_source(i, step, ex1, ey1, ez1);
        if (!la) { zero(ex1); zero(ey1); zero(ez1); zero(hx); zero(hy); zero(hz); }
        if (own && la && i >= T.i0 && i < T.i1) record(i, c, step, ex1, ey1, ez1, hx, hy, hz);
        stv<V>(&L1x[tq], ex1);
        stv<V>(&L1z[tq], ez1);
        if (lane == 0) { Se1[rr][seg][0] = ex1[0]; Se1[rr][seg][1] = ey1[0]; }

        if (PF) prefetch(i + 1);
        // ---- step 2 at plane ib = i-1 (H on the halo row above too) ----
        const int ib = i - 1;
        const bool pb = ib >= ia && rr <= T.nrows && rok;  // wave-uniform
        const bool wb = own && rok && ib >= T.i0;          // E too, and stored
        const unsigned cq = ((unsigned)(pb ? ib : 0) * ny + jr) * nz + kb;
        const AxP Xp = prof(p.x, pb ? ib : 0, ikx, jkx);
        const bool inx2 = PXY && pb && ok && Xp.s >= 0, iny2 = PXY && pb && ok && Y.s >= 0;
        const unsigned qx2 = inx2 ? xs3(Xp.s, j, kb, ny, nz) : 0, qy2 = iny2 ? ys3(ib, Y.s, kb, sy, nz) : 0;
        float hx2[V], hy2[V], hz2[V];
#pragma unroll
        for (int v = 0; v < V; ++v) { hx2[v] = hx1p[v]; hy2[v] = hy1p[v]; hz2[v] = hz1p[v]; }
        if (pb) {  // wave-uniform
            const bool sn2 = last && seamnext;
            const float exs = sn2 ? e1s[0] : 0.f, eys = sn2 ? e1s[1] : 0.f;
            float q2[4][V];  // x/y-slab psi of H at (ib, j): n+1 in, n+2 out
            if (PXY) qload(q2, PM, PSI_HXY, PSI_HZY, PSI_HYX, PSI_HZX, qy2, iny2, qx2, inx2);
            hstep(hx2, hy2, hz2, dbp, ex1p, ey1p, ez1p, ey1, ez1, ex1y, ez1y, exs, eys, dyz, dxz, Xp, Y, inx2, iny2, q2);
            if (PXY && wb) qstore(q2, P1, PSI_HXY, PSI_HZY, PSI_HYX, PSI_HZX, qy2, iny2, qx2, inx2);
            if (PZ && zany) {
                float p1[V], p2[V];
                zstash_r(p1, ib & 1, 0);
                zstash_r(p2, ib & 1, 1);
                hfix(hx2, hy2, dbp, dyz, dxz, p1, p2, true, true);
                if (wb) {
                    zout(0, p1);
                    zout(1, p2);
                }
            }
        }
        if (!SB) __syncthreads();  // step-1 LDS reads of this plane are done
        stv<V>(&H2x[tq], hx2);
        stv<V>(&H2z[tq], hz2);
        if (lane == 63) { Sh2[rr][seg][0] = hx2[V - 1]; Sh2[rr][seg][1] = hy2[V - 1]; }
        __syncthreads();
        if (wb) {  // wave-uniform
            float hxj2[V], hzj2[V];
            zero(hxj2);
            zero(hzj2);
            if (jm) {
                ldv<V>(hxj2, &H2x[tq - ROW]);
                ldv<V>(hzj2, &H2z[tq - ROW]);
            }
            const float hxs2 = (lane == 0 && seg > 0) ? Sh2[rr][seg > 0 ? seg - 1 : 0][0] : 0.f;
            const float hys2 = (lane == 0 && seg > 0) ? Sh2[rr][seg > 0 ? seg - 1 : 0][1] : 0.f;
            float e2x[V], e2y[V], e2z[V];
#pragma unroll
            for (int v = 0; v < V; ++v) { e2x[v] = ex1p[v]; e2y[v] = ey1p[v]; e2z[v] = ez1p[v]; }
            float e2q[4][V];  // x/y-slab psi of E at (ib, j): n+1 in, n+2 out
            if (PXY) qload(e2q, PM, PSI_EXY, PSI_EZY, PSI_EYX, PSI_EZX, qy2, iny2, qx2, inx2);
            estep(e2x, e2y, e2z, cap, cbp, hx2, hy2, hz2, hy2p, hz2p, hxj2, hzj2, hxs2, hys2, ib >= 1, dyz, dxz, Xp, Y,
                  inx2, iny2, e2q);
            if (PXY) qstore(e2q, P1, PSI_EXY, PSI_EZY, PSI_EYX, PSI_EZX, qy2, iny2, qx2, inx2);
            if (PZ && zany) {  // zany implies ok
                float p3[V], p4[V];
                zstash_r(p3, ib & 1, 2);
                zstash_r(p4, ib & 1, 3);
                efix(e2x, e2y, cbp, dyz, dxz, p3, p4, ib >= 1);
                zout(2, p3);
                zout(3, p4);
            }
            add_source(ib, step + 1, e2x, e2y, e2z);
            record(ib, cq, step + 1, e2x, e2y, e2z, hx2, hy2, hz2);
            if (ok) {
                stv<V>(p.s1.f[FDTD_EX] + cq, e2x);
                stv<V>(p.s1.f[FDTD_EY] + cq, e2y);
                stv<V>(p.s1.f[FDTD_EZ] + cq, e2z);
                stv<V>(p.s1.f[FDTD_HX] + cq, hx2);
                stv<V>(p.s1.f[FDTD_HY] + cq, hy2);
                stv<V>(p.s1.f[FDTD_HZ] + cq, hz2);
            }
        }
        // ---- carry ----
#pragma unroll
        for (int v = 0; v < V; ++v) {
            eyc[v] = eyx[v];
            ezc[v] = ezx[v];
            hx1p[v] = hx[v]; hy1p[v] = hy[v]; hz1p[v] = hz[v];
            ex1p[v] = ex1[v]; ey1p[v] = ey1[v]; ez1p[v] = ez1[v];
            hy2p[v] = hy2[v]; hz2p[v] = hz2[v];
            cbp[v] = cb[v]; cap[v] = ca[v]; dbp[v] = db[v];
        }
    }
    if (PZ && iend - 1 >= T.i0) {
        __syncthreads();
        zflush(iend - 1);
    }
}

template <int V, int RZ, int R, bool PZ, bool PXY, int MAT, bool REC, int SL>
__global__ __launch_bounds__(64 * RZ * (R + 2)) void k3d_two(Prob3D p, const TileTB *tiles, ProbeTiles pt,
                                                           int64_t step, State3D mid) {
    constexpr int NR = R + 2, NT = 64 * RZ * NR, ZW = kTwoZMax + 8, NZR = NR + 1;
    constexpr bool SB = two_sb(PXY, MAT, NR * RZ);
    __shared__ float LEx[NT * V], LEz[NT * V], LHx[NT * V], LHz[NT * V], L1x[NT * V], L1z[NT * V];
    __shared__ float LH2x[SB ? NT * V : 1], LH2z[SB ? NT * V : 1];
    __shared__ float Se0[NR][RZ][2], Sh1[NR][RZ][2], Se1[NR][RZ][2], Sh2[NR][RZ][2];
    __shared__ __align__(16) float ZT[PZ ? 6 : 1][PZ ? ZW : 4];
    __shared__ __align__(16) float ZP[PZ ? 4 : 1][PZ ? NZR * ZW : 4];
    __shared__ __align__(16) float Zs[PZ ? 2 : 1][PZ ? NR : 1][PZ ? 4 : 1][PZ ? ZW : 4];
    __shared__ __align__(16) float ZQ[PZ ? 4 : 1][PZ ? R * ZW : 4];
    TwoLds<V, RZ, R, PZ, SB> L{LEx, LEz, LHx, LHz, L1x, L1z, LH2x, LH2z, Se0, Sh1, Se1, Sh2, ZT, ZP, Zs, ZQ};
    const int tix = xcd_block(blockIdx.x, gridDim.x);
    const TileTB T = tiles[tix];
    if (T.i0 >= T.i1) return;  // padding
    if constexpr (SL == 4) {
        // tiles near x slabs only or y slabs only: the code path of the
        // tile's kind (wave-uniform), the register allocation of the larger
        const int a = max(T.i0 - 2, 0), b = min(T.i1, p.nx - 1);
        const bool onx = (p.x.lo > 0 && a < p.x.lo) || (p.x.hi > 0 && b >= p.nx - p.x.hi);
        if (onx) two_tile<V, RZ, R, PZ, PXY, MAT, REC, 1>(p, T, tix, pt, step, mid, L);
        else two_tile<V, RZ, R, PZ, PXY, MAT, REC, 2>(p, T, tix, pt, step, mid, L);
    } else {
        two_tile<V, RZ, R, PZ, PXY, MAT, REC, SL>(p, T, tix, pt, step, mid, L);
    }
}

// REC: the instance holds the probe read-out.  Without x/y-slab code a
// launch with no probe entries (pt.start == nullptr) runs the instance
// without it: the read-out code, even where no tile executes it, made the
// plane loop 4 % slower.  SL: slab kinds of the x/y-slab instance (3 both,
// 4 one kind per tile, by a code path each; 0 without x/y-slab code).
template <int RZ, bool PZ, bool PXY, int MAT, bool REC, int SL>
static void go_two(const Prob3D &p, const TileTB *tiles, int n, const ProbeTiles &pt, int64_t step,
                   const State3D &mid, hipStream_t st) {
    constexpr int W = two_waves(PZ, MAT, PXY), R = W / RZ - 2;
    hipLaunchKernelGGL((k3d_two<4, RZ, R, PZ, PXY, MAT, REC, SL>), dim3((unsigned)n), dim3(64 * W), 0, st, p, tiles,
                       pt, step, mid);
}

template <int RZ, bool PZ, bool PXY, bool REC, int SL>
static void go_two_m(const Prob3D &p, const TileTB *tiles, int n, const ProbeTiles &pt, int64_t step,
                     const State3D &mid, hipStream_t st) {
    const int mat = p.db ? 2 : (p.ca ? 1 : 0);
    if (mat == 0) go_two<RZ, PZ, PXY, 0, REC, SL>(p, tiles, n, pt, step, mid, st);
    else if (mat == 1) go_two<RZ, PZ, PXY, 1, REC, SL>(p, tiles, n, pt, step, mid, st);
    else go_two<RZ, PZ, PXY, 2, REC, SL>(p, tiles, n, pt, step, mid, st);
}

template <int RZ, bool PZ>
static void go_two_s(const Prob3D &p, const TileTB *tiles, int n, const ProbeTiles &pt, int64_t step,
                     const State3D &mid, int slab, hipStream_t st) {
    if (slab == 4) go_two_m<RZ, PZ, true, true, 4>(p, tiles, n, pt, step, mid, st);
    else go_two_m<RZ, PZ, true, true, 3>(p, tiles, n, pt, step, mid, st);
}

template <int RZ>
static void go_two_c(const Prob3D &p, const TileTB *tiles, int n, const ProbeTiles &pt, int64_t step,
                     const State3D *mid, int slab, hipStream_t st) {
    const bool pz = p.z.lo + p.z.hi > 0;
    if (mid) {
        if (pz) go_two_s<RZ, true>(p, tiles, n, pt, step, *mid, slab, st);
        else go_two_s<RZ, false>(p, tiles, n, pt, step, *mid, slab, st);
    } else {
        const State3D none{};
        if (pt.start) {
            if (pz) go_two_m<RZ, true, false, true, 0>(p, tiles, n, pt, step, none, st);
            else go_two_m<RZ, false, false, true, 0>(p, tiles, n, pt, step, none, st);
        } else {
            if (pz) go_two_m<RZ, true, false, false, 0>(p, tiles, n, pt, step, none, st);
            else go_two_m<RZ, false, false, false, 0>(p, tiles, n, pt, step, none, st);
        }
    }
}

hipError_t launch_3d_two(const Prob3D &p, const TileTB *tiles, int n, const ProbeTiles &pt, int64_t step,
                         hipStream_t st, const State3D *mid, int slab) {
    if (n <= 0) return hipSuccess;
    if (!two3d_supported(p.nx, p.ny, p.nz, p.z.lo, p.z.hi)) return hipErrorInvalidValue;
    if (mid && p.x.lo + p.x.hi + p.y.lo + p.y.hi > 0) {
        // the slab psi arrays of the middle state must exist
        for (int a : {PSI_HXY, PSI_HZY, PSI_EXY, PSI_EZY})
            if (p.y.lo + p.y.hi > 0 && !mid->psi[a]) return hipErrorInvalidValue;
        for (int a : {PSI_HYX, PSI_HZX, PSI_EYX, PSI_EZX})
            if (p.x.lo + p.x.hi > 0 && !mid->psi[a]) return hipErrorInvalidValue;
    }
    if (slab != 3 && slab != 4) return hipErrorInvalidValue;
    if (p.nz <= 64 * 4) go_two_c<1>(p, tiles, n, pt, step, mid, slab, st);
    else go_two_c<2>(p, tiles, n, pt, step, mid, slab, st);
    return hipGetLastError();
}

}  // namespace gem
