// Discrete adjoint of the 2D TMz step (transposed message passing run
// backward in time).  One backward step applies the transpose of the E
// layer, then the transpose of the H layer, to the adjoint state
// (lEz, lHx, lHy and the adjoint CPML values), as three in-place gather
// kernels:
//   A: per cell, E layer^T pointwise: probe-loss seed, u = Cb*a,
//      gx/gy temporaries, adjoint psi_E, gradient, lEz <- Ca*a
//   B: per cell, gather gx/gy into lHx/lHy, then H layer^T pointwise:
//      ex/ey temporaries and adjoint psi_H
//   C: per cell, gather ex/ey into lEz
// (E layer^T: each E node sends Cb-weighted messages back to the H nodes it
// gathered from; H layer^T likewise back to the E nodes.)  The 1/d factors
// are folded in the axis tables exactly as in the forward kernels.
#include "common.hpp"

namespace gem {

struct AdjArgs {
    Prob2D p;          // forward problem (coefficients, axis tables)
    Adj2D a;
    int4 design;       // [i0,i1) x [j0,j1)
    const float *cap_ez;   // Ez^k at design cells (before the E layer of step k)
    const float *cap_br;   // bracket of the E layer of step k at design cells
    const float *dca, *dcb;
    double *grad;
    // probe-loss seed: lEz[probe] += 2 * Ez^{k+1}[probe] when k+1 in (n0, n1]
    int seed_on;
    const int *pb_start;   // per block of 256 cells: probe entries
    const int *pb_cell;
    const int *pb_slot;
    const float *rec;      // forward probe record [np][rec_stride]
    int64_t rec_stride;
    int64_t k;
};

__global__ __launch_bounds__(256) void k_adj_a(AdjArgs A) {
    const Prob2D &p = A.p;
    const int64_t n = (int64_t)p.nx * p.ny;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    const int ny = p.ny;
    const int i = (int)(c / ny), j = (int)(c - (int64_t)i * ny);
    float a = A.a.ez[c];
    if (A.seed_on) {
        const int b0 = A.pb_start[blockIdx.x], b1 = A.pb_start[blockIdx.x + 1];
        for (int q = b0; q < b1; ++q)
            if (A.pb_cell[q] == c) a += 2.f * A.rec[(int64_t)A.pb_slot[q] * A.rec_stride + A.k];
    }
    float gx = 0.f, gy = 0.f;
    if (i >= 1 && j >= 1) {
        const float u = p.cb[c] * a;
        const int ii = slab_index(p.x, i), jj = slab_index(p.y, j);
        const int sy = p.y.lo + p.y.hi;
        float px = u, py = -u;
        if (ii >= 0) {
            float *q = A.a.psi_ezx + (int64_t)ii * ny + j;
            px += *q;
            *q = p.x.bE[i] * px;
        }
        if (jj >= 0) {
            float *q = A.a.psi_ezy + (int64_t)i * sy + jj;
            py += *q;
            *q = p.y.bE[j] * py;
        }
        gy = u * p.x.kE[i] + p.x.cE[i] * px;
        gx = -u * p.y.kE[j] + p.y.cE[j] * py;
        if (i >= A.design.x && i < A.design.y && j >= A.design.z && j < A.design.w) {
            const int64_t q = (int64_t)(i - A.design.x) * (A.design.w - A.design.z) + (j - A.design.z);
            A.grad[q] += (double)a * ((double)A.dca[q] * A.cap_ez[q] + (double)A.dcb[q] * A.cap_br[q]);
        }
        a *= p.ca ? p.ca[c] : 1.f;
    }
    A.a.gx[c] = gx;
    A.a.gy[c] = gy;
    A.a.ez[c] = a;
}

__global__ __launch_bounds__(256) void k_adj_b(AdjArgs A) {
    const Prob2D &p = A.p;
    const int64_t n = (int64_t)p.nx * p.ny;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    const int ny = p.ny;
    const int i = (int)(c / ny), j = (int)(c - (int64_t)i * ny);
    float hy = A.a.hy[c] + A.a.gy[c] - ((i + 1 < p.nx) ? A.a.gy[c + ny] : 0.f);
    float hx = A.a.hx[c] + A.a.gx[c] - ((j + 1 < ny) ? A.a.gx[c + 1] : 0.f);
    const float db = p.db ? p.db[c] : p.db0;
    const int ii = slab_index(p.x, i), jj = slab_index(p.y, j);
    const int sy = p.y.lo + p.y.hi;
    // Hx: forward Hx -= Db (kH dEy + psi), psi <- b psi + c dEy
    float wx = -db * hx;
    if (jj >= 0) {
        float *q = A.a.psi_hx + (int64_t)i * sy + jj;
        wx += *q;
        *q = p.y.bH[j] * wx;
    }
    const float ey = -db * hx * p.y.kH[j] + p.y.cH[j] * wx;
    // Hy: forward Hy += Db (kH dEx + psi)
    float wy = db * hy;
    if (ii >= 0) {
        float *q = A.a.psi_hy + (int64_t)ii * ny + j;
        wy += *q;
        *q = p.x.bH[i] * wy;
    }
    const float ex = db * hy * p.x.kH[i] + p.x.cH[i] * wy;
    A.a.hx[c] = hx;
    A.a.hy[c] = hy;
    A.a.ex[c] = ex;
    A.a.ey[c] = ey;
}

__global__ __launch_bounds__(256) void k_adj_c(AdjArgs A) {
    const Prob2D &p = A.p;
    const int64_t n = (int64_t)p.nx * p.ny;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    const int ny = p.ny;
    const int i = (int)(c / ny), j = (int)(c - (int64_t)i * ny);
    float v = A.a.ez[c] - A.a.ey[c] - A.a.ex[c];
    if (j >= 1) v += A.a.ey[c - 1];
    if (i >= 1) v += A.a.ex[c - ny];
    A.a.ez[c] = v;
}

__global__ void k_grad_to_float(const double *g, float *out, int64_t n) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) out[q] = (float)g[q];
}

hipError_t launch_adj2d(const Prob2D &p, const Adj2D &a, int64_t k, const int *design,
                        const float *cap_ez, const float *cap_br, const float *dca,
                        const float *dcb, double *grad, int seed_on, const int *pb_start,
                        const int *pb_cell, const int *pb_slot, const float *rec,
                        int64_t rec_stride, hipStream_t st) {
    AdjArgs A;
    A.p = p;
    A.a = a;
    A.design = make_int4(design[0], design[1], design[2], design[3]);
    A.cap_ez = cap_ez;
    A.cap_br = cap_br;
    A.dca = dca;
    A.dcb = dcb;
    A.grad = grad;
    A.seed_on = seed_on;
    A.pb_start = pb_start;
    A.pb_cell = pb_cell;
    A.pb_slot = pb_slot;
    A.rec = rec;
    A.rec_stride = rec_stride;
    A.k = k;
    const int64_t n = (int64_t)p.nx * p.ny;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_adj_a, dim3(nb), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_adj_b, dim3(nb), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_adj_c, dim3(nb), dim3(256), 0, st, A);
    return hipGetLastError();
}

hipError_t launch_grad_to_float(const double *g, float *out, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_to_float, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, out, n);
    return hipGetLastError();
}

}  // namespace gem
