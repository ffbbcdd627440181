// Explicit-graph form: one CSR gather per layer (Prop. 2: h_l = sum over the
// neighbourhood of w * h).  Rows are the nodes a layer updates; weights are
// the fixed coefficients.  Gather only (each row written by one thread, its
// edges summed in order), so results are deterministic.
#include "common.hpp"

namespace gem {

// One wavefront per 64 consecutive rows.  Its edge range [rowptr[r0],
// rowptr[r0 + 64]) is staged in LDS by coalesced loads; each lane then sums
// its row from LDS in edge order (a segment longer than the staging space
// reads memory directly, same order).  A row of at most 8 edges (every row
// of the FDTD graphs) issues all its gathers before the first product, so
// they are in flight together instead of one per loop trip (4096^2 TMz
// graph: 24.6 -> 29.1 Gcell/s); the sum keeps the edge order.
constexpr int kCsrCap = 512;  // staged edges per wavefront

__global__ __launch_bounds__(256) void k_csr_layer(const int *__restrict__ rowptr,
                                                   const int *__restrict__ col,
                                                   const float *__restrict__ w,
                                                   const int *__restrict__ dst, const float *x,
                                                   float *y, int nrows) {
    __shared__ int sc[4][kCsrCap];
    __shared__ float sw[4][kCsrCap];
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = (int)(threadIdx.x & 63);
    const int r0 = ((int)blockIdx.x * 4 + wv) * 64;
    const int r = r0 + lane;
    const bool live = r0 < nrows;  // wave-uniform
    int b0 = 0, n = 0, b = 0, e = 0;
    if (live) {
        const int rl = min(r0 + 64, nrows);
        b0 = rowptr[r0];
        n = rowptr[rl] - b0;
        if (r < nrows) {
            b = rowptr[r];
            e = rowptr[r + 1];
        }
        if (n <= kCsrCap)
            for (int q = lane; q < n; q += 64) {
                sc[wv][q] = col[b0 + q];
                sw[wv][q] = w[b0 + q];
            }
    }
    __syncthreads();
    if (!live || r >= nrows) return;
    float acc = 0.f;
    if (n <= kCsrCap && e - b <= 8) {
        const int q0 = b - b0, len = e - b;
        float wq[8], xq[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            wq[u] = u < len ? sw[wv][q0 + u] : 0.f;
            xq[u] = u < len ? x[sc[wv][q0 + u]] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (u < len) acc += wq[u] * xq[u];
    } else if (n <= kCsrCap) {
        for (int q = b - b0; q < e - b0; ++q) acc += sw[wv][q] * x[sc[wv][q]];  // longer rows (none in the graphs built here)
    } else {
        for (int q = b; q < e; ++q) acc += w[q] * x[col[q]];
    }
    y[dst[r]] = acc;
}

hipError_t launch_csr_layer(const int *rowptr, const int *col, const float *w, const int *dst,
                            const float *x, float *y, int nrows, hipStream_t st) {
    if (nrows <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((nrows + 255) / 256);
    hipLaunchKernelGGL(k_csr_layer, dim3(nb), dim3(256), 0, st, rowptr, col, w, dst, x, y, nrows);
    return hipGetLastError();
}

// Soft source on its nodes, then probe samples (one block).
__global__ void k_node_src_probe(float *x, const int *src_nodes, int nsrc, const float *src_vals,
                                 int64_t src_len, int64_t step, int np, const int *probe_node,
                                 const int *probe_node2, float *rec, int64_t rec_stride, int64_t rec_index) {
    if (step < src_len)
        for (int q = threadIdx.x; q < nsrc; q += blockDim.x) x[src_nodes[q]] += src_vals[step];
    __syncthreads();
    for (int q = threadIdx.x; q < np; q += blockDim.x)
        rec[(int64_t)q * rec_stride + rec_index] = x[probe_node[q]] + (probe_node2 ? x[probe_node2[q]] : 0.f);
}

hipError_t launch_node_source_probe(float *x, const int *src_nodes, int nsrc, const float *src_vals,
                                    int64_t src_len, int64_t step, int np,
                                    const int *probe_node, const int *probe_node2, float *rec, int64_t rec_stride,
                                    int64_t rec_index, hipStream_t st) {
    if (nsrc <= 0 && np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_node_src_probe, dim3(1), dim3(256), 0, st, x, src_nodes, nsrc, src_vals, src_len,
                       step, np, probe_node, probe_node2, rec, rec_stride, rec_index);
    return hipGetLastError();
}

}  // namespace gem
