// Explicit-graph form: one CSR gather per layer (Prop. 2: h_l = sum over the
// neighbourhood of w * h).  Rows are the nodes a layer updates; weights are
// the fixed coefficients.  Gather only (each row written by one thread, its
// edges summed in order), so results are deterministic.
#include "common.hpp"
#include "devutil.hpp"

namespace gem {

// One wavefront per 64 consecutive rows.  Its edge range [rowptr[r0],
// rowptr[r0 + 64]) is staged in LDS by coalesced loads; each lane then sums
// its row from LDS in edge order (a segment longer than the staging space
// reads memory directly, same order).  A row of at most 8 edges (every row
// without an auxiliary group) issues all its gathers before the first
// product, so they are in flight together instead of one per loop trip
// (4096^2 TMz graph: 24.6 -> 29.1 Gcell/s); the sum keeps the edge order.
// An auxiliary group (a CPML psi row that only this row reads, stored
// inside the row behind a marker edge) is summed in place, stored at its
// node and weighted by the marker: one launch per layer, and its edges come
// with the row's own (one dependent gather, not three).  Rows whose
// destinations step evenly (all but the chunks that straddle a grid row)
// take them from the chunk table, not from dst.
constexpr int kCsrCap = 640;  // staged edges per wavefront (20 KB per workgroup)

// the row's sum, edges [q, q + len) read through col_at / w_at
template <class C, class Wt>
__device__ __forceinline__ float csr_row_groups(float *x, int q, int len, C col_at, Wt w_at) {
    float acc = 0.f, s = 0.f, wm = 0.f;
    int rem = 0, node = 0;
    for (int u = 0; u < len; ++u) {
        const int c = col_at(q + u);
        const float w = w_at(q + u);
        if (rem > 0) {  // inside an auxiliary group: its first edge is its own node
            const float v = x[c];
            if (node < 0) node = c;
            s += w * v;
            if (--rem == 0) {
                x[node] = s;
                acc += wm * s;
            }
        } else if (c < 0) {
            rem = -1 - c;
            wm = w;
            s = 0.f;
            node = -1;
        } else {
            acc += w * x[c];
        }
    }
    return acc;
}

__global__ __launch_bounds__(256) void k_csr_layer(CsrLayerArgs L, float *x) {
    __shared__ int sc[4][kCsrCap];
    __shared__ float sw[4][kCsrCap];
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = (int)(threadIdx.x & 63);
    const int nrows = L.nrows;
    // the slab rows recur at a fixed stride in row order: in plain
    // round-robin they would fall on the same XCDs (the H layer of a
    // 4096-wide grid: all on two of the eight; 627 -> 563 us per step)
    const int r0 = (xcd_scatter((int)blockIdx.x, (int)gridDim.x) * 4 + wv) * 64;
    const int r = r0 + lane;
    const bool live = r0 < nrows;  // wave-uniform
    // {first destination, stride (0: dst[]), rows with auxiliary groups}
    const int4 ch = live ? L.chunk[r0 >> 6] : make_int4(0, 0, 0, 0);
    int b0 = 0, n = 0, b = 0, e = 0;
    if (live) {
        const int rl = min(r0 + 64, nrows);
        b0 = L.rowptr[r0];
        n = L.rowptr[rl] - b0;
        if (r < nrows) {
            b = L.rowptr[r];
            e = L.rowptr[r + 1];
        }
        if (n <= kCsrCap)
            for (int q = lane; q < n; q += 64) {
                sc[wv][q] = L.col[b0 + q];
                sw[wv][q] = L.w[b0 + q];
            }
    }
    __syncthreads();
    if (!live || r >= nrows) return;
    float acc = 0.f;
    const int q0 = b - b0, len = e - b;
    if (n <= kCsrCap && !ch.z && len <= 8) {
        float wq[8], xq[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            wq[u] = u < len ? sw[wv][q0 + u] : 0.f;
            xq[u] = u < len ? x[sc[wv][q0 + u]] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (u < len) acc += wq[u] * xq[u];
    } else if (n <= kCsrCap && len <= 16) {
        // auxiliary groups: every node value first (in flight together),
        // then the sums in edge order
        float xq[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = u < len ? sc[wv][q0 + u] : -1;
            xq[u] = c >= 0 ? x[c] : 0.f;
        }
        float s = 0.f, wm = 0.f;
        int rem = 0, node = 0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            if (u < len) {
                const int c = sc[wv][q0 + u];
                const float w = sw[wv][q0 + u];
                if (rem > 0) {  // inside a group: its first edge is its own node
                    if (node < 0) node = c;
                    s += w * xq[u];
                    if (--rem == 0) {
                        x[node] = s;
                        acc += wm * s;
                    }
                } else if (c < 0) {
                    rem = -1 - c;
                    wm = w;
                    s = 0.f;
                    node = -1;
                } else {
                    acc += w * xq[u];
                }
            }
        }
    } else if (n <= kCsrCap) {  // longer rows (none in the graphs built here)
        acc = csr_row_groups(x, q0, len, [&](int q) { return sc[wv][q]; }, [&](int q) { return sw[wv][q]; });
    } else {
        acc = csr_row_groups(x, b, len, [&](int q) { return L.col[q]; }, [&](int q) { return L.w[q]; });
    }
    x[ch.y != 0 ? ch.x + (r - r0) * ch.y : L.dst[r]] = acc;
}

hipError_t launch_csr_layer(const CsrLayerArgs &L, float *x, hipStream_t st) {
    if (L.nrows <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((L.nrows + 255) / 256);
    hipLaunchKernelGGL(k_csr_layer, dim3(nb), dim3(256), 0, st, L, x);
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
