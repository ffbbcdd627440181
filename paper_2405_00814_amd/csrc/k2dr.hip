// Whole small 2D grid in one workgroup (kernel variant 4 for 2D grids): the
// state stays in registers for all the steps of an fdtd_step call, and the
// two layers of every step (Eq. 8-9, then Eq. 7, in TMz form; Prop. 2) are
// separated by workgroup barriers instead of kernel launches.  A step of a
// grid this small costs about one dependent launch in the other variants;
// here it costs its arithmetic on one CU and two barriers.
//
// 1024 threads: the columns j of a row band are consecutive lanes (bands
// start on a wavefront, ny rounded up to 64 lanes); a thread holds the Ez,
// Hx, Hy and Cb of up to 16 rows of its column (Ca in LDS).  Neighbours:
// j+1 and j-1 from the DPP lane shifts, across a wavefront edge from a
// column of the neighbouring wavefront in LDS; i+1 and i-1 from the
// thread's own rows, across a band edge from the neighbouring band's first
// or last row in LDS.  No CPML (PEC walls: the E layer leaves row 0 and
// column 0, the H layer reads Ez beyond the last row and column as 0), no
// mu_r map (uniform Db).
// Soft source after the E layer; probes sample after the step.
#include <algorithm>

#include "common.hpp"
#include "devutil.hpp"

namespace gem {

namespace {

constexpr int kResThreads = 1024, kResRows = 16, kResProbes = 64;

struct ResLayout {
    int nyp, nbk, rb;  // lanes per band (ny rounded up to 64), bands, rows per band
};

__host__ __device__ inline ResLayout res_layout(int nx, int ny) {
    ResLayout L{};
    L.nyp = (ny + 63) / 64 * 64;
    L.nbk = L.nyp <= kResThreads ? kResThreads / L.nyp : 0;
    L.rb = L.nbk > 0 ? (nx + L.nbk - 1) / L.nbk : 0;
    return L;
}

}  // namespace

// RR: rows held per thread (4, 8 or 16: the band's rows rounded up)
template <int MAT, int RR>
__global__ __launch_bounds__(kResThreads) void k2d_resident(Prob2D p, int64_t step0, int nsteps) {
    const int nx = p.nx, ny = p.ny;
    const ResLayout L = res_layout(nx, ny);
    const int t = (int)threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int b = t / L.nyp, j = t - b * L.nyp;
    const int i0 = b * L.rb;
    const int nr = b < L.nbk ? max(0, min(L.rb, nx - i0)) : 0;  // rows of this band (<= RR)
    const bool col = j < ny && nr > 0;
    // wavefront neighbours in the same band (their columns continue this
    // one's): the next wavefront's first lane, the previous one's last
    const bool wnext = col && ((w + 1) * 64) % L.nyp != 0, wprev = col && (w * 64) % L.nyp != 0;
    const int wn = min(w + 1, kResThreads / 64 - 1), wp = max(w - 1, 0);  // seam rows (read on every lane)
    const bool e63 = wnext && j + 1 < ny;
    __shared__ float sEz[kResThreads / 64][RR];  // lane 0's Ez, per wavefront
    __shared__ float sHx[kResThreads / 64][RR];  // lane 63's Hx, per wavefront
    __shared__ float sEzR[kResThreads];          // band's first-row Ez, per band and column
    __shared__ float sHyR[kResThreads];          // band's last-row Hy
    __shared__ int sPr[kResProbes], sNext[kResProbes];  // probe q: its row, the holder's next probe
    __shared__ int sFirst[kResThreads];                 // a thread's first probe (-1: none)
    // Ca map in LDS (row r of thread t at r * 1024 + t): in registers as
    // well it would make the kernel spill
    __shared__ float sCa[MAT >= 1 ? RR * kResThreads : 1];
    const float jkx = p.x.kE[0], jky = p.y.kE[0];
    const float dbx = p.db0 * p.x.kH[0], dby = p.db0 * p.y.kH[0];  // the H layer's weights

    // Cb = 0, Ca = 1 where the E layer leaves Ez as it is (row 0, column 0,
    // and the lanes and rows outside the grid): the update then needs no
    // per-cell condition
    float ez[RR], hx[RR], hy[RR], cb[RR];  // Ca: sCa
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const bool in = col && r < nr;
        const bool upd = in && i0 + r >= 1 && j >= 1;
        const int64_t c = (int64_t)(i0 + r) * ny + j;
        ez[r] = in ? p.s0.ez[c] : 0.f;
        hx[r] = in ? p.s0.hx[c] : 0.f;
        hy[r] = in ? p.s0.hy[c] : 0.f;
        cb[r] = upd ? p.cb[c] : 0.f;
        if (MAT >= 1) sCa[MAT >= 1 ? r * kResThreads + t : 0] = (upd && p.ca) ? p.ca[c] : 1.f;
    }
    // probes: a list per thread holding probe cells (first in sFirst,
    // then sNext), built once; the thread keeps its first in a register
    const int np = min(p.np, kResProbes);
    sFirst[t] = -1;
    __syncthreads();
    if (t < np) {
        const int cell = p.probe_idx[t];
        const int pi = cell / ny, pj = cell - pi * ny;
        sPr[t] = pi % L.rb;
        sNext[t] = atomicExch(&sFirst[pi / L.rb * L.nyp + pj], t);
    }
    __syncthreads();
    const int myq = sFirst[t];
    auto pick = [&](const float (&a)[RR], int r) {
        float v = 0.f;
#pragma unroll
        for (int u = 0; u < RR; ++u) v = u == r ? a[u] : v;
        return v;
    };
    const int *sb = p.src_box;
    const bool scol = p.src_idx >= 0 && col && (unsigned)(j - sb[2]) < (unsigned)(sb[3] - sb[2]);

    // E^n seams for the first H layer
    if (lane == 0)
#pragma unroll
        for (int r = 0; r < RR; ++r) sEz[w][r] = ez[r];
    sEzR[t] = ez[0];
    __syncthreads();
    // the source value of each step is loaded at the start of the step
    // before (its latency then overlaps that step's work)
    float sv = (scol && step0 < p.src_len) ? p.src_vals[step0] : 0.f;
    for (int s = 0; s < nsteps; ++s) {
        const int64_t n = step0 + s;
        const float svn = (scol && s + 1 < nsteps && n + 1 < p.src_len) ? p.src_vals[n + 1] : 0.f;
        // ---- H layer: Ez(i, j+1), Ez(i+1, j) ----
        const float elast = (b + 1 < L.nbk && i0 + nr < nx) ? sEzR[t + L.nyp] : 0.f;  // Ez of row i0 + nr
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            // the lane shift runs on every lane (a shift inside one arm of
            // the select would read a disabled lane there)
            const float sh = lane_next(ez[r]);
            const float seam = sEz[wn][r];  // same address on every lane
            const float en = lane == 63 ? (e63 ? seam : 0.f) : sh;
            const float es = r + 1 < nr ? ez[r + 1 < RR ? r + 1 : r] : elast;
            hx[r] -= dby * (en - ez[r]);
            hy[r] += dbx * (es - ez[r]);
        }
        // H seams for the E layer
        if (lane == 63)
#pragma unroll
            for (int r = 0; r < RR; ++r) sHx[w][r] = hx[r];
        sHyR[t] = nr == RR ? hy[RR - 1] : pick(hy, nr - 1);  // uniform
        __syncthreads();
        // ---- E layer: Hx(i, j-1), Hy(i-1, j) ----
        const float hfirst = b > 0 ? sHyR[t - L.nyp] : 0.f;  // Hy of row i0 - 1
        const bool srcn = scol && n < p.src_len;
        const float sval = sv;
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const int i = i0 + r;
            const float sh = lane_prev(hx[r]);
            const float seam = sHx[wp][r];
            const float hw = lane == 0 ? (wprev ? seam : 0.f) : sh;
            const float hn = r > 0 ? hy[r > 0 ? r - 1 : 0] : hfirst;
            const float tx = (hy[r] - hn) * jkx;
            const float ty = (hx[r] - hw) * jky;
            ez[r] = (MAT >= 1 ? sCa[MAT >= 1 ? r * kResThreads + t : 0] * ez[r] : ez[r]) + cb[r] * (tx - ty);
            if (srcn && r < nr && (unsigned)(i - sb[0]) < (unsigned)(sb[1] - sb[0])) ez[r] += sval;
        }
        // probes (after the step), by the thread holding the cell
        for (int q = myq; q >= 0; q = sNext[q]) {
            const int r = sPr[q];
            float v;
            if (p.probe_comp == FDTD_HX) v = pick(hx, r);  // uniform
            else if (p.probe_comp == FDTD_HY) v = pick(hy, r);
            else v = pick(ez, r);
            p.rec[(int64_t)q * p.rec_stride + (n - p.rec_base)] = v;
        }
        // E seams for the next H layer
        if (lane == 0)
#pragma unroll
            for (int r = 0; r < RR; ++r) sEz[w][r] = ez[r];
        sEzR[t] = ez[0];
        sv = svn;
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < RR; ++r)
        if (col && r < nr) {
            const int64_t c = (int64_t)(i0 + r) * ny + j;
            p.s1.ez[c] = ez[r];
            p.s1.hx[c] = hx[r];
            p.s1.hy[c] = hy[r];
        }
}

bool res2d_supported(int nx, int ny, bool cpml, int np) {
    if (cpml || nx < 1 || ny < 1) return false;
    const ResLayout L = res_layout(nx, ny);
    return L.nbk >= 1 && L.rb <= kResRows && np <= kResProbes;
}

template <int MAT>
static void launch_rr(const Prob2D &q, int rb, int64_t step, int k, hipStream_t st) {
    if (rb <= 4) hipLaunchKernelGGL((k2d_resident<MAT, 4>), dim3(1), dim3(kResThreads), 0, st, q, step, k);
    else if (rb <= 8) hipLaunchKernelGGL((k2d_resident<MAT, 8>), dim3(1), dim3(kResThreads), 0, st, q, step, k);
    else hipLaunchKernelGGL((k2d_resident<MAT, 16>), dim3(1), dim3(kResThreads), 0, st, q, step, k);
}

hipError_t launch_2d_resident(const Prob2D &p, int mat, int64_t step, int64_t nsteps, hipStream_t st) {
    if (nsteps <= 0) return hipSuccess;
    if (p.ezy || p.db || mat < 0 || mat > 1) return hipErrorInvalidValue;
    for (int64_t done = 0; done < nsteps;) {
        // at most 2^16 steps per launch
        const int k = (int)std::min<int64_t>(nsteps - done, 65536);
        Prob2D q = p;
        if (done > 0) q.s0 = p.s1;  // later launches continue in place
        const int rb = res_layout(p.nx, p.ny).rb;
        if (rb > kResRows) return hipErrorInvalidValue;
        if (mat == 0) launch_rr<0>(q, rb, step + done, k, st);
        else launch_rr<1>(q, rb, step + done, k, st);
        done += k;
    }
    return hipGetLastError();
}

}  // namespace gem
