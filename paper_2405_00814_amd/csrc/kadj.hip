// Discrete adjoint of the 2D TMz step (transposed message passing run
// backward in time).  One backward step applies the transpose of the E
// layer, then the transpose of the H layer, to the adjoint state (lEz, lHx,
// lHy and the adjoint CPML values), in three phases per cell:
//   A: E layer^T pointwise: u = Cb*a (a = lEz with the probe-loss seed),
//      messages gx, gy to the H nodes, adjoint psi_E, gradient, lEz <- Ca*a
//   B: gather gx/gy into lHx/lHy, then H layer^T pointwise: messages ex, ey
//      to the E nodes and adjoint psi_H
//   C: gather ex/ey into lEz
// (E layer^T: each E node sends Cb-weighted messages back to the H nodes it
// gathered from; H layer^T likewise back to the E nodes.)  The 1/d factors
// are folded in the axis tables exactly as in the forward kernels.
#include "common.hpp"
#include "devutil.hpp"

namespace gem {

// ---------------------------------------------------------------------------
// Fused adjoint step: the three phases above in one pass over memory, by the
// forward kernel's tiling (a wavefront marches TX rows of a 64*V column
// strip).  Double buffered: the adjoint state of step k+1 is read from L0,
// that of step k written to L1.  At row i the wavefront has phase A of rows i
// (carried) and i+1, phase B of rows i-1 (carried) and i, and writes row i.
// The strip's edge columns take their neighbours' values by recomputation:
// lanes 0 and 63 hold the neighbouring strips' edge columns and recompute
// them (phase B needs phase A's gx at j+1, phase C phase B's ey at j-1), so
// a strip owns the 62*V columns of lanes 1..62 and no lane waits on a
// scalar recompute.  The probe-loss seed of the next step is added to the
// written adjoint Ez by the cell's owner.
// ---------------------------------------------------------------------------
struct AdjFArgs {
    Prob2D p;
    Adj2D l0, l1;      // adjoint state read (step k+1) and written (step k)
    int4 design;
    // captured values of this step on the box cbox (the design box and one
    // row and column beyond it, clipped to the grid): Ez before the E layer
    // and the E layer's bracket, row width cw
    int4 cbox;
    int cw;
    const float *cap_ez, *cap_br;
    // per design cell: sez += a Ez^n, sbr += a bracket (the gradients with
    // respect to any per-cell parameter of Ca and Cb follow from these two
    // sums and the coefficients' derivatives)
    double *sez, *sbr;
    // with the mu_r gradient (nullptr: none), per design cell: shx += aHx bx,
    // shy += aHy by, the H layer's brackets rebuilt from the captured Ez
    // (the design box is clear of the CPML slabs: no auxiliary term)
    double *shx, *shy;
    // probe-loss seed of the next step, added to the written adjoint Ez:
    // l1.ez[probe] += 2 * rec[slot][seed_k] (probes grouped by tile, entries
    // of one cell consecutive)
    int seed_out;
    ProbeTiles pt;
    const float *rec;
    int64_t rec_stride, seed_k;
};

template <int V>
__device__ __forceinline__ void ldva(float (&r)[V], const float *p) {
    if constexpr (V == 4) {
        const float4 t = *reinterpret_cast<const float4 *>(p);
        r[0] = t.x; r[1] = t.y; r[2] = t.z; r[3] = t.w;
    } else if constexpr (V == 2) {
        const float2 t = *reinterpret_cast<const float2 *>(p);
        r[0] = t.x; r[1] = t.y;
    } else {
        r[0] = *p;
    }
}

template <int V>
__device__ __forceinline__ void stva(float *p, const float (&r)[V]) {
    if constexpr (V == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(r[0], r[1], r[2], r[3]);
    } else if constexpr (V == 2) {
        *reinterpret_cast<float2 *>(p) = make_float2(r[0], r[1]);
    } else {
        *p = r[0];
    }
}

template <int V, bool PML>
__global__ __launch_bounds__(256) void k_adj_fused(AdjFArgs A, int TX, int nsy, int ntiles) {
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int tw = ((nb % 8 == 0) ? (b % 8) * (nb / 8) + (b / 8) : b) * 4 + (int)(threadIdx.x >> 6);
    if (tw >= ntiles) return;  // whole wavefront leaves; no barriers below
    const Prob2D &p = A.p;
    const Adj2D &L0 = A.l0, &L1 = A.l1;
    const int lane = threadIdx.x & 63;
    const int nx = p.nx, ny = p.ny;
    const int cx = tw / nsy, sy = tw - cx * nsy;
    const int x0 = cx * TX, x1 = min(x0 + TX, nx);
    const int jb = sy * 62 * V - V + lane * V;       // lane 0: the column group left of the strip
    const bool valid = jb >= 0 && jb < ny;           // ny % V == 0
    const bool own = valid && lane >= 1 && lane <= 62;
    const int syw = p.y.lo + p.y.hi;
    const int dw = A.design.w - A.design.z;

    float kEy[V], bEy[V], cEy[V], kHy[V], bHy[V], cHy[V];
    int jj[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int j = valid ? jb + v : 0;
        kEy[v] = p.y.kE[j]; kHy[v] = p.y.kH[j];
        bEy[v] = p.y.bE[j]; cEy[v] = p.y.cE[j];
        bHy[v] = p.y.bH[j]; cHy[v] = p.y.cH[j];
        jj[v] = (PML && valid) ? slab_index(p.y, j) : -1;
    }
    auto zero = [](float (&a)[V]) {
#pragma unroll
        for (int v = 0; v < V; ++v) a[v] = 0.f;
    };
    // phase A of row i (own columns): gx, gy messages, Ca-weighted adjoint
    // Ez; writes the new E-type psi and the gradient when `write`
    auto phaseA = [&](int i, float (&gx)[V], float (&gy)[V], float (&aca)[V], bool wr) {
        const bool write = wr && own;
        zero(gx); zero(gy); zero(aca);
        if (i < 0 || i >= nx || !valid) return;
        const int64_t row = (int64_t)i * ny;
        float a[V], cb[V], ca[V];
        ldva<V>(a, L0.ez + row + jb);
        ldva<V>(cb, p.cb + row + jb);
        if (p.ca) ldva<V>(ca, p.ca + row + jb);
        else {
#pragma unroll
            for (int v = 0; v < V; ++v) ca[v] = 1.f;
        }
        const int ii = PML ? slab_index(p.x, i) : -1;
        const float kEx = p.x.kE[i], bEx = p.x.bE[i], cEx = p.x.cE[i];
        float px_o[V], px_n[V];
        if (PML && ii >= 0) ldva<V>(px_o, L0.psi_ezx + (int64_t)ii * ny + jb);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int j = jb + v;
            aca[v] = a[v];
            if (PML && ii >= 0) px_n[v] = px_o[v];
            if (i >= 1 && j >= 1) {
                const float u = cb[v] * a[v];
                float px = u, py = -u;
                if (PML && ii >= 0) {
                    px += px_o[v];
                    px_n[v] = bEx * px;
                }
                if (PML && jj[v] >= 0) {
                    const int64_t q = (int64_t)i * syw + jj[v];
                    py += L0.psi_ezy[q];
                    if (write) L1.psi_ezy[q] = bEy[v] * py;
                }
                gy[v] = u * kEx + cEx * px;
                gx[v] = -u * kEy[v] + cEy[v] * py;
                if (write && i >= A.design.x && i < A.design.y && j >= A.design.z && j < A.design.w) {
                    const int64_t q = (int64_t)(i - A.design.x) * dw + (j - A.design.z);
                    const int64_t qc = (int64_t)(i - A.cbox.x) * A.cw + (j - A.cbox.z);
                    A.sez[q] += (double)a[v] * A.cap_ez[qc];
                    A.sbr[q] += (double)a[v] * A.cap_br[qc];
                }
                aca[v] = a[v] * ca[v];
            } else if (PML && jj[v] >= 0 && write) {
                const int64_t q = (int64_t)i * syw + jj[v];
                L1.psi_ezy[q] = L0.psi_ezy[q];
            }
        }
        if (PML && ii >= 0 && write) stva<V>(L1.psi_ezx + (int64_t)ii * ny + jb, px_n);
    };
    // prologue: A of row x0, ex of row x0-1
    float gx_c[V], gy_c[V], aca_c[V], ex_p[V];
    phaseA(x0, gx_c, gy_c, aca_c, true);
    zero(ex_p);
    if (x0 >= 1 && valid) {
        const int i = x0 - 1;
        const int64_t row = (int64_t)i * ny;
        float gxm[V], gym[V], acam[V], hy[V], db[V];
        phaseA(i, gxm, gym, acam, false);
        ldva<V>(hy, L0.hy + row + jb);
        if (p.db) ldva<V>(db, p.db + row + jb);
        else {
#pragma unroll
            for (int v = 0; v < V; ++v) db[v] = p.db0;
        }
        const int ii = PML ? slab_index(p.x, i) : -1;
        float py_o[V];
        if (PML && ii >= 0) ldva<V>(py_o, L0.psi_hy + (int64_t)ii * ny + jb);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const float h = hy[v] + gym[v] - gy_c[v];
            float wy = db[v] * h;
            if (PML && ii >= 0) wy += py_o[v];
            ex_p[v] = db[v] * h * p.x.kH[i] + p.x.cH[i] * wy;
        }
    }

    // the tile's probe entries for the loss seed, read once
    const int qs0 = A.seed_out ? A.pt.start[tw] : 0, qs1 = A.seed_out ? A.pt.start[tw + 1] : 0;
    for (int i = x0; i < x1; ++i) {
        const int64_t row = (int64_t)i * ny;
        float gx_n[V], gy_n[V], aca_n[V];
        phaseA(i + 1, gx_n, gy_n, aca_n, i + 1 < x1);
        // gx at j+1
        float gxr[V];
#pragma unroll
        for (int v = 0; v + 1 < V; ++v) gxr[v] = gx_c[v + 1];
        gxr[V - 1] = lane_next(gx_c[0]);  // lane 63: not needed
        // ---- phase B (H layer transposed) ----
        float hx[V], hy[V], db[V], ex[V], ey[V];
        zero(hx); zero(hy); zero(ex); zero(ey);
#pragma unroll
        for (int v = 0; v < V; ++v) db[v] = p.db0;
        const int ii = PML ? slab_index(p.x, i) : -1;
        if (valid) {
            ldva<V>(hx, L0.hx + row + jb);
            ldva<V>(hy, L0.hy + row + jb);
            if (p.db) ldva<V>(db, p.db + row + jb);
            float py_o[V], py_n[V];
            if (PML && ii >= 0) ldva<V>(py_o, L0.psi_hy + (int64_t)ii * ny + jb);
            const float kHx = p.x.kH[i], bHx = p.x.bH[i], cHx = p.x.cH[i];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                hy[v] = hy[v] + gy_c[v] - gy_n[v];
                hx[v] = hx[v] + gx_c[v] - gxr[v];
                float wx = -db[v] * hx[v];
                if (PML && jj[v] >= 0) {
                    const int64_t q = (int64_t)i * syw + jj[v];
                    wx += L0.psi_hx[q];
                    if (own) L1.psi_hx[q] = bHy[v] * wx;
                }
                ey[v] = -db[v] * hx[v] * kHy[v] + cHy[v] * wx;
                float wy = db[v] * hy[v];
                if (PML && ii >= 0) {
                    wy += py_o[v];
                    py_n[v] = bHx * wy;
                }
                ex[v] = db[v] * hy[v] * kHx + cHx * wy;
            }
            // mu_r gradient at the design cells: hx, hy are now the
            // adjoints of H after this step's H layer
            if (A.shx && own && i >= A.design.x && i < A.design.y) {
                const int64_t r0 = (int64_t)(i - A.cbox.x) * A.cw;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int j = jb + v;
                    if (j < A.design.z || j >= A.design.w) continue;
                    const int64_t q = (int64_t)(i - A.design.x) * dw + (j - A.design.z);
                    const int64_t qc = r0 + (j - A.cbox.z);
                    const float e0 = A.cap_ez[qc];
                    const float ey1 = j + 1 < A.cbox.w ? A.cap_ez[qc + 1] : 0.f;
                    const float ex1 = i + 1 < A.cbox.y ? A.cap_ez[qc + A.cw] : 0.f;
                    A.shx[q] += (double)hx[v] * (double)((ey1 - e0) * kHy[v]);
                    A.shy[q] += (double)hy[v] * (double)((ex1 - e0) * kHx);
                }
            }
            if (own) {
                stva<V>(L1.hx + row + jb, hx);
                stva<V>(L1.hy + row + jb, hy);
                if (PML && ii >= 0) stva<V>(L1.psi_hy + (int64_t)ii * ny + jb, py_n);
            }
        }
        // ey at j-1
        float eyl[V];
#pragma unroll
        for (int v = 1; v < V; ++v) eyl[v] = ey[v - 1];
        eyl[0] = lane_prev(ey[V - 1]);  // lane 0: not needed
        // ---- phase C (gather into adjoint Ez) ----
        if (own) {
            float ez[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                float w = aca_c[v] - ey[v] - ex[v];
                if (jb + v >= 1) w += eyl[v];
                if (i >= 1) w += ex_p[v];
                ez[v] = w;
            }
            if (qs0 < qs1) {
                for (int q = qs0; q < qs1; ++q) {
                    const int c = A.pt.cell[q];
                    const int pi = c / ny, pj = c - pi * ny;
                    if (pi != i) continue;
                    const float add = 2.f * A.rec[(int64_t)A.pt.slot[q] * A.rec_stride + A.seed_k];
#pragma unroll
                    for (int v = 0; v < V; ++v) ez[v] = pj == jb + v ? ez[v] + add : ez[v];
                }
            }
            stva<V>(L1.ez + row + jb, ez);
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            gx_c[v] = gx_n[v]; gy_c[v] = gy_n[v]; aca_c[v] = aca_n[v]; ex_p[v] = ex[v];
        }
    }
}

// probe-loss seed: lEz[probe] += 2 * Ez^{k+1}[probe]; one thread per probed
// cell (entries sorted by cell, [start[u], start[u+1]) share cell u), so
// probes sharing a cell add up in order
__global__ void k_adj_seed(float *ez, const int *start, const int *cell, const int *slot, int nu,
                           const float *rec, int64_t rec_stride, int64_t k) {
    const int u = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (u >= nu) return;
    const int q0 = start[u], q1 = start[u + 1];
    const int c = cell[q0];
    float v = ez[c];
    for (int q = q0; q < q1; ++q) v += 2.f * rec[(int64_t)slot[q] * rec_stride + k];
    ez[c] = v;
}

hipError_t launch_adj2d_seed(float *ez, const int *seed_start, const int *seed_cell, const int *seed_slot, int nu,
                             const float *rec, int64_t rec_stride, int64_t k, hipStream_t st) {
    if (nu <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_seed, dim3((unsigned)((nu + 63) / 64)), dim3(64), 0, st, ez, seed_start, seed_cell,
                       seed_slot, nu, rec, rec_stride, k);
    return hipGetLastError();
}

hipError_t launch_adj2d_fused(const Prob2D &p, const Adj2D &l0, const Adj2D &l1, const int *design,
                              const int *cbox, const float *cap_ez, const float *cap_br, double *sez, double *sbr,
                              double *shx, double *shy, int seed_out, const ProbeTiles &pt, const float *rec,
                              int64_t rec_stride, int64_t seed_k, int V, int TX, hipStream_t st) {
    if (p.ny % V != 0 || TX < 1) return hipErrorInvalidValue;
    AdjFArgs A;
    A.seed_out = seed_out;
    A.pt = pt;
    A.rec = rec;
    A.rec_stride = rec_stride;
    A.seed_k = seed_k;
    A.p = p;
    A.l0 = l0;
    A.l1 = l1;
    A.design = make_int4(design[0], design[1], design[2], design[3]);
    A.cbox = make_int4(cbox[0], cbox[1], cbox[2], cbox[3]);
    A.cw = cbox[3] - cbox[2];
    A.shx = shx;
    A.shy = shy;
    A.cap_ez = cap_ez;
    A.cap_br = cap_br;
    A.sez = sez;
    A.sbr = sbr;
    const int nsy = (p.ny + 62 * V - 1) / (62 * V), ncx = (p.nx + TX - 1) / TX;
    const int nt = nsy * ncx;
    const dim3 g((unsigned)((nt + 3) / 4)), b(256);
    const bool pml = p.x.lo + p.x.hi + p.y.lo + p.y.hi > 0;
#define GEM_A(VV)                                                                                   \
    do {                                                                                            \
        if (pml) hipLaunchKernelGGL((k_adj_fused<VV, true>), g, b, 0, st, A, TX, nsy, nt);        \
        else hipLaunchKernelGGL((k_adj_fused<VV, false>), g, b, 0, st, A, TX, nsy, nt);           \
    } while (0)
    switch (V) {
        case 1: GEM_A(1); break;
        case 2: GEM_A(2); break;
        case 4: GEM_A(4); break;
        default: return hipErrorInvalidValue;
    }
#undef GEM_A
    return hipGetLastError();
}

__global__ void k_grad_combine(const double *sez, const double *sbr, const double *dca, const double *dcb,
                               float *out, int64_t n) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) out[q] = (float)(dca[q] * sez[q] + dcb[q] * sbr[q]);
}

hipError_t launch_grad_combine(const double *sez, const double *sbr, const double *dca, const double *dcb, float *out,
                               int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sez, sbr, dca, dcb, out,
                       n);
    return hipGetLastError();
}

}  // namespace gem
