// 2D TMz: TB leapfrog steps per pass over memory (temporal blocking).
//
// One wavefront is one tile: x rows [i0, i1) of a strip of 64 lanes x V
// consecutive y columns.  The HL = ceil(TB / V) lanes at each side of the
// strip hold the neighbouring tiles' columns and are recomputed, so the
// strip's own columns are exact after TB steps (the valid width shrinks by
// one column per side and step: the H layer reads Ez at j+1, the E layer Hx
// at j-1).  The wavefront marches along x through a pipeline of TB stages
// held in registers: at iteration t stage k (0-based) advances row t-k from
// state n+k to n+k+1, using
//   - state n+k of rows t-k and t-k+1: stage k-1's output of the previous
//     and of the current iteration (stage 0: state n from memory);
//   - its own Hy of row t-k-1 from the previous iteration.
// Only the last stage's rows [i0, i1) of the own columns are written, so
// tiles are independent: no LDS, no barriers, no atomics.  Rows below i0
// enter the pipeline TB rows early (recomputed like the halo columns), rows
// from i1 on TB-1 rows late.  Arithmetic per cell is that of the single-step
// kernel, in the same order.
#include "common.hpp"
#include "devutil.hpp"

namespace gem {

// Per stage: the state of one row (fields, coefficients, CPML psi).
template <int V>
struct Row2 {
    float e[V], hx[V], hy[V];
    float cb[V], ca[V], db[V];
    float phx[V], pezy[V];  // y-slab psi (H-type, E-type)
    float phy[V], pezx[V];  // x-slab psi
};

// MAT: 0 = Cb map; 1 = Ca and Cb maps; 2 = Ca, Cb and Db maps.
// PML: CPML code (tiles whose cone touches a slab); BATCH: the tile names
// its problem in `probs` and the step is read from step_base.
template <int V, int TB, bool PML, int MAT, bool BATCH>
__global__ __launch_bounds__(256) void k2d_tb(Prob2D p1, const Prob2D *__restrict__ probs,
                                              const Tile2T *__restrict__ tiles, int ntiles, ProbeTiles pt,
                                              const int64_t *__restrict__ step_base, int64_t step0,
                                              CapArgs cap) {
    constexpr int HL = (TB + V - 1) / V;  // halo lanes per side
    constexpr int OW = (64 - 2 * HL) * V;  // own columns per strip
    // the wavefront's tile index, uniform across its lanes: read once as a
    // scalar, so the tile, its problem and the row loop bounds stay scalar
    // (as per-lane values they held 10-30 more VGPRs per lane and made the
    // row loop divergent)
    const int tw = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    if (tw >= ntiles) return;  // whole wavefront leaves; no barriers below
    const Tile2T T = tiles[tw];
    const Prob2D &p = BATCH ? probs[T.prob] : p1;
    const int64_t step = (BATCH ? *step_base : 0) + step0;
    const int lane = threadIdx.x & 63;
    const int nx = p.nx, ny = p.ny;
    const int jb = T.ja - HL * V + lane * V;  // first column of the lane
    const bool valid = jb >= 0 && jb < ny;    // ny % V == 0: all V columns or none
    const bool own = valid && lane >= HL && lane < 64 - HL;
    const int syw = p.y.lo + p.y.hi;
    (void)OW;

    // y profile of the lane's columns (interior value without PML code)
    float kHy[V], kEy[V], bHy[V], cHy[V], bEy[V], cEy[V];
    int jj[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int j = valid ? jb + v : p.y.lo;
        kHy[v] = PML ? p.y.kH[j] : p.y.kH[p.y.lo];
        kEy[v] = PML ? p.y.kE[j] : p.y.kE[p.y.lo];
        jj[v] = -1;
        bHy[v] = cHy[v] = bEy[v] = cEy[v] = 0.f;
        if (PML && valid) {
            jj[v] = slab_index(p.y, j);
            if (jj[v] >= 0) {
                bHy[v] = p.y.bH[j]; cHy[v] = p.y.cH[j];
                bEy[v] = p.y.bE[j]; cEy[v] = p.y.cE[j];
            }
        }
    }
    const float kHx0 = p.x.kH[p.x.lo], kEx0 = p.x.kE[p.x.lo];
    float sval[TB];
#pragma unroll
    for (int k = 0; k < TB; ++k) sval[k] = (p.src_idx >= 0 && step + k < p.src_len) ? p.src_vals[step + k] : 0.f;
    // the source box, read once (the batched instances read p from memory):
    // an empty box without a source
    const bool hs = p.src_idx >= 0;
    const int si0 = hs ? p.src_box[0] : 0, si1 = hs ? p.src_box[1] : 0, sj0 = p.src_box[2], sj1 = p.src_box[3];

    auto zero = [](float (&a)[V]) {
#pragma unroll
        for (int v = 0; v < V; ++v) a[v] = 0.f;
    };
    // everything but Ez
    auto clear_row = [&](Row2<V> &r) {
        zero(r.hx); zero(r.hy); zero(r.cb); zero(r.phx); zero(r.pezy); zero(r.phy); zero(r.pezx);
#pragma unroll
        for (int v = 0; v < V; ++v) { r.ca[v] = 1.f; r.db[v] = p.db0; }
    };
    // state n of row i except Ez (fields, coefficients, psi)
    auto load_row = [&](Row2<V> &r, int i) {
        clear_row(r);
        if (i < 0 || i >= nx || !valid) return;
        const int64_t row = (int64_t)i * ny + jb;
        ldv<V>(r.hx, p.s0.hx + row);
        ldv<V>(r.hy, p.s0.hy + row);
        ldv<V>(r.cb, p.cb + row);
        if (MAT >= 1 && p.ca) ldv<V>(r.ca, p.ca + row);
        if (MAT == 2 && p.db) ldv<V>(r.db, p.db + row);
        if (PML) {
            const int ii = slab_index(p.x, i);
            if (ii >= 0) {
                ldv<V>(r.phy, p.s0.psi_hy + (int64_t)ii * ny + jb);
                ldv<V>(r.pezx, p.s0.psi_ezx + (int64_t)ii * ny + jb);
            }
#pragma unroll
            for (int v = 0; v < V; ++v)
                if (jj[v] >= 0) {
                    r.phx[v] = p.s0.psi_hx[(int64_t)i * syw + jj[v]];
                    r.pezy[v] = p.s0.psi_ezy[(int64_t)i * syw + jj[v]];
                }
        }
    };
    auto load_ez = [&](float (&e)[V], int i) {
        zero(e);
        if (i >= 0 && i < nx && valid) ldv<V>(e, p.s0.ez + (int64_t)i * ny + jb);
    };

    Row2<V> in[TB];      // stage k's input: state n+k of row t-k
    float hyp[TB][V];    // stage k's Hy of row t-k-1
#pragma unroll
    for (int k = 0; k < TB; ++k) {
        clear_row(in[k]);
        zero(in[k].e);
        zero(hyp[k]);
    }
    const int t0 = T.i0 - TB, t1 = T.i1 + TB - 1;
    // the tile's probe entries, read once (not at every stage: the stage
    // would wait for the load to decide its loop)
    const int pbeg = pt.start != nullptr ? pt.start[tw] : 0, pend = pt.start != nullptr ? pt.start[tw + 1] : 0;
    load_ez(in[0].e, t0);
    // Single-problem instances without CPML code load stage 0's memory
    // input of the next iteration (Ez^n of row t+1, the rest of state n of
    // row t) one iteration ahead, so the loads overlap the stages'
    // arithmetic (measured 3-7 % faster with one and four columns per lane,
    // even with two).  The CPML instances load at the top of the iteration
    // (the extra registers would cost them a wavefront per SIMD), and so do
    // the batched ones (measured 3 % slower with the prefetch).
    constexpr bool PF = !PML && !BATCH;
    float en_nx[V];
    Row2<V> r_nx;
    if (PF) {
        load_ez(en_nx, t0 + 1);
        load_row(r_nx, t0);
    }

    for (int t = t0; t < t1; ++t) {
        float en0[V];
        if (PF) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                en0[v] = en_nx[v];
                in[0].hx[v] = r_nx.hx[v]; in[0].hy[v] = r_nx.hy[v];
                in[0].cb[v] = r_nx.cb[v]; in[0].ca[v] = r_nx.ca[v]; in[0].db[v] = r_nx.db[v];
                in[0].phx[v] = r_nx.phx[v]; in[0].pezy[v] = r_nx.pezy[v];
                in[0].phy[v] = r_nx.phy[v]; in[0].pezx[v] = r_nx.pezx[v];
            }
            if (t + 1 < t1) {
                load_ez(en_nx, t + 2);
                load_row(r_nx, t + 1);
            }
        } else {
            load_ez(en0, t + 1);
            load_row(in[0], t);
        }
        Row2<V> out, prev;
        clear_row(prev);
        zero(prev.e);
#pragma unroll
        for (int k = 0; k < TB; ++k) {
            const int i = t - k;
            const bool rv = i >= 0 && i < nx;
            const Row2<V> &a = in[k];
            float en[V];
#pragma unroll
            for (int v = 0; v < V; ++v) en[v] = k == 0 ? en0[v] : prev.e[v];
            const float kHx = PML && rv ? p.x.kH[i] : kHx0, kEx = PML && rv ? p.x.kE[i] : kEx0;
            const int ii = (PML && rv) ? slab_index(p.x, i) : -1;
            float bHx = 0.f, cHx = 0.f, bEx = 0.f, cEx = 0.f;
            if (PML && ii >= 0) { bHx = p.x.bH[i]; cHx = p.x.cH[i]; bEx = p.x.bE[i]; cEx = p.x.cE[i]; }
            // Ez(i, j+1)
            float er[V];
#pragma unroll
            for (int v = 0; v + 1 < V; ++v) er[v] = a.e[v + 1];
            er[V - 1] = lane_next(a.e[0]);
            // ---- H layer ----
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const float dEy = er[v] - a.e[v];
                float ty = dEy * kHy[v];
                out.phx[v] = a.phx[v];
                if (PML && jj[v] >= 0) {
                    out.phx[v] = bHy[v] * a.phx[v] + cHy[v] * dEy;
                    ty += out.phx[v];
                }
                out.hx[v] = a.hx[v] - a.db[v] * ty;
                const float dEx = en[v] - a.e[v];
                float tx = dEx * kHx;
                out.phy[v] = a.phy[v];
                if (PML && ii >= 0) {
                    out.phy[v] = bHx * a.phy[v] + cHx * dEx;
                    tx += out.phy[v];
                }
                out.hy[v] = a.hy[v] + a.db[v] * tx;
            }
            // Hx(i, j-1)
            float hl[V];
#pragma unroll
            for (int v = 1; v < V; ++v) hl[v] = out.hx[v - 1];
            hl[0] = lane_prev(out.hx[V - 1]);
            const bool mine = own && i >= T.i0 && i < T.i1;
            // design-cell capture (single problem): Ez before the E layer
            // and the E layer's bracket, per step
            const bool capi = !BATCH && cap.ez != nullptr && mine && i >= cap.design.x && i < cap.design.y;
            // ---- E layer ----
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int j = jb + v;
                out.e[v] = a.e[v];
                out.pezx[v] = a.pezx[v];
                out.pezy[v] = a.pezy[v];
                if (i >= 1 && j >= 1) {
                    const float dHy = out.hy[v] - hyp[k][v];
                    const float dHx = out.hx[v] - hl[v];
                    float tx = dHy * kEx;
                    float ty = dHx * kEy[v];
                    if (PML && ii >= 0) {
                        out.pezx[v] = bEx * a.pezx[v] + cEx * dHy;
                        tx += out.pezx[v];
                    }
                    if (PML && jj[v] >= 0) {
                        out.pezy[v] = bEy[v] * a.pezy[v] + cEy[v] * dHx;
                        ty += out.pezy[v];
                    }
                    out.e[v] = (MAT >= 1 ? a.ca[v] * a.e[v] : a.e[v]) + a.cb[v] * (tx - ty);
                    if (capi && j >= cap.design.z && j < cap.design.w) {
                        const int64_t q = (step + k - cap.k0) * cap.nd + (int64_t)(i - cap.design.x) *
                                          (cap.design.w - cap.design.z) + (j - cap.design.z);
                        cap.ez[q] = a.e[v];
                        cap.br[q] = tx - ty;
                    }
                }
                if ((unsigned)(i - si0) < (unsigned)(si1 - si0) && (unsigned)(j - sj0) < (unsigned)(sj1 - sj0))
                    out.e[v] += sval[k];
            }
            // outside the grid: the ghost values are zero
            if (!rv || !valid) {
                zero(out.e); zero(out.hx); zero(out.hy);
                zero(out.phx); zero(out.pezy); zero(out.phy); zero(out.pezx);
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                out.cb[v] = a.cb[v]; out.ca[v] = a.ca[v]; out.db[v] = a.db[v];
                hyp[k][v] = out.hy[v];
            }
            // probes of this tile, state n+k+1
            if (pbeg < pend && mine) {
                for (int q = pbeg; q < pend; ++q) {
                    const int cell = pt.cell[q];
                    const int pi = cell / ny, pj = cell - pi * ny;
                    if (pi != i) continue;
                    float val = 0.f;
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const float x = p.probe_comp == FDTD_HX ? out.hx[v]
                                      : p.probe_comp == FDTD_HY ? out.hy[v] : out.e[v];
                        val = pj == jb + v ? x : val;
                    }
                    if (pj >= jb && pj < jb + V)
                        p.rec[(int64_t)pt.slot[q] * p.rec_stride + (step + k - p.rec_base)] = val;
                }
            }
            if (k == TB - 1) {
                if (mine) {
                    const int64_t row = (int64_t)i * ny + jb;
                    stv<V>(p.s1.ez + row, out.e);
                    stv<V>(p.s1.hx + row, out.hx);
                    stv<V>(p.s1.hy + row, out.hy);
                    if (PML) {
                        if (ii >= 0) {
                            stv<V>(p.s1.psi_hy + (int64_t)ii * ny + jb, out.phy);
                            stv<V>(p.s1.psi_ezx + (int64_t)ii * ny + jb, out.pezx);
                        }
#pragma unroll
                        for (int v = 0; v < V; ++v)
                            if (jj[v] >= 0) {
                                p.s1.psi_hx[(int64_t)i * syw + jj[v]] = out.phx[v];
                                p.s1.psi_ezy[(int64_t)i * syw + jj[v]] = out.pezy[v];
                            }
                    }
                }
            }
            // stage k is done with in[k]: it takes stage k-1's output of this
            // iteration (state n+k of row t-k+1) for the next one
            if (k > 0) in[k] = prev;
            prev = out;
        }
        // stage 0 of the next iteration starts from Ez^n of row t+1
#pragma unroll
        for (int v = 0; v < V; ++v) in[0].e[v] = en0[v];
    }
}

template <int V, int TB, bool PML, int MAT>
static void go_tb(const Prob2D &p, const Prob2D *probs, const Tile2T *tiles, int n, const ProbeTiles &pt,
                  const int64_t *step_base, int64_t step, const CapArgs &cap, hipStream_t st) {
    const dim3 g((unsigned)((n + 3) / 4)), b(256);
    if (probs)
        hipLaunchKernelGGL((k2d_tb<V, TB, PML, MAT, true>), g, b, 0, st, p, probs, tiles, n, pt, step_base, step,
                           cap);
    else
        hipLaunchKernelGGL((k2d_tb<V, TB, PML, MAT, false>), g, b, 0, st, p, probs, tiles, n, pt, step_base, step,
                           cap);
}

template <int V, int TB>
static void go_tb_m(const Prob2D &p, const Prob2D *probs, const Tile2T *tiles, int n, bool pml, int mat,
                    const ProbeTiles &pt, const int64_t *step_base, int64_t step, const CapArgs &cap,
                    hipStream_t st) {
#define GEM_TB(PM, MA) go_tb<V, TB, PM, MA>(p, probs, tiles, n, pt, step_base, step, cap, st)
    if (pml) {
        if (mat == 0) GEM_TB(true, 0);
        else if (mat == 1) GEM_TB(true, 1);
        else GEM_TB(true, 2);
    } else {
        if (mat == 0) GEM_TB(false, 0);
        else if (mat == 1) GEM_TB(false, 1);
        else GEM_TB(false, 2);
    }
#undef GEM_TB
}

hipError_t launch_2d_tb(const Prob2D &p, const Prob2D *probs_dev, const Tile2T *tiles, int ntiles, bool pml,
                        int mat, const ProbeTiles &pt, int V, int TB, const int64_t *step_base, int64_t step,
                        hipStream_t st, const CapArgs *capture) {
    if (ntiles <= 0) return hipSuccess;
    if (capture && probs_dev) return hipErrorInvalidValue;
    CapArgs cap{};
    if (capture) cap = *capture;
    if (!probs_dev && p.ny % V != 0) return hipErrorInvalidValue;
    if (mat < 0 || mat > 2) return hipErrorInvalidValue;
    if (V == 1 && TB == 2) go_tb_m<1, 2>(p, probs_dev, tiles, ntiles, pml, mat, pt, step_base, step, cap, st);
    else if (V == 1 && TB == 4) go_tb_m<1, 4>(p, probs_dev, tiles, ntiles, pml, mat, pt, step_base, step, cap, st);
    else if (V == 2 && TB == 2) go_tb_m<2, 2>(p, probs_dev, tiles, ntiles, pml, mat, pt, step_base, step, cap, st);
    else if (V == 2 && TB == 4) go_tb_m<2, 4>(p, probs_dev, tiles, ntiles, pml, mat, pt, step_base, step, cap, st);
    else if (V == 4 && TB == 2) go_tb_m<4, 2>(p, probs_dev, tiles, ntiles, pml, mat, pt, step_base, step, cap, st);
    else if (V == 4 && TB == 4) go_tb_m<4, 4>(p, probs_dev, tiles, ntiles, pml, mat, pt, step_base, step, cap, st);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace gem
