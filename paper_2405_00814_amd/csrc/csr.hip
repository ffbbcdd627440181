// Explicit-graph form: one CSR gather per layer (Prop. 2: h_l = sum over the
// neighbourhood of w * h).  Rows are the nodes a layer updates; weights are
// the fixed coefficients.  Gather only (each row written by one thread), so
// results are deterministic.
#include "common.hpp"

namespace gem {

__global__ __launch_bounds__(256) void k_csr_layer(const int *__restrict__ rowptr,
                                                   const int *__restrict__ col,
                                                   const float *__restrict__ w,
                                                   const int *__restrict__ dst, const float *x,
                                                   float *y, int nrows) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const int b = rowptr[r], e = rowptr[r + 1];
    float acc = 0.f;
    for (int q = b; q < e; ++q) acc += w[q] * x[col[q]];
    y[dst[r]] = acc;
}

hipError_t launch_csr_layer(const int *rowptr, const int *col, const float *w, const int *dst,
                            const float *x, float *y, int nrows, hipStream_t st) {
    if (nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_csr_layer, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, st,
                       rowptr, col, w, dst, x, y, nrows);
    return hipGetLastError();
}

// Soft source on one node, then probe samples (one block).
__global__ void k_node_src_probe(float *x, int64_t src_node, const float *src_vals,
                                 int64_t src_len, int64_t step, int np, const int *probe_node,
                                 float *rec, int64_t rec_stride, int64_t rec_index) {
    if (threadIdx.x == 0 && src_node >= 0 && step < src_len) x[src_node] += src_vals[step];
    __syncthreads();
    for (int q = threadIdx.x; q < np; q += blockDim.x)
        rec[(int64_t)q * rec_stride + rec_index] = x[probe_node[q]];
}

hipError_t launch_node_source_probe(float *x, int64_t src_node, const float *src_vals,
                                    int64_t src_len, int64_t step, int np,
                                    const int *probe_node, float *rec, int64_t rec_stride,
                                    int64_t rec_index, hipStream_t st) {
    if (src_node < 0 && np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_node_src_probe, dim3(1), dim3(64), 0, st, x, src_node, src_vals, src_len,
                       step, np, probe_node, rec, rec_stride, rec_index);
    return hipGetLastError();
}

}  // namespace gem
