// 3D Yee kernels: the H layer gathers the curl of E into Hx, Hy, Hz, the E
// layer gathers the curl of H into Ex, Ey, Ez (the paper's Eq. 7-9 extended
// to six components, which Sec. IV-A states carries over directly), with
// CPML auxiliary values in the boundary slabs.
#include "common.hpp"

namespace gem {

__device__ __forceinline__ int64_t xs_idx(int ii, int j, int k, int ny, int nz) {
    return ((int64_t)ii * ny + j) * nz + k;
}
__device__ __forceinline__ int64_t ys_idx(int i, int jj, int k, int sy, int nz) {
    return ((int64_t)i * sy + jj) * nz + k;
}
__device__ __forceinline__ int64_t zs_idx(int i, int j, int kk, int ny, int sz) {
    return ((int64_t)i * ny + j) * sz + kk;
}

// psi <- b psi + c D at a slab cell; returns the new value.
__device__ __forceinline__ float cpml_upd(const float *src, float *dst, int64_t q, float b,
                                          float c, float D) {
    const float ps = b * src[q] + c * D;
    dst[q] = ps;
    return ps;
}

// ---------------------------------------------------------------------------
// Two-pass reference kernels (one thread per cell, in place on s0)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k3d_ref_h(Prob3D p) {
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int k = (int)(c % nz);
    const int j = (int)((c / nz) % ny);
    const int i = (int)(c / ((int64_t)ny * nz));
    const int64_t sxs = (int64_t)ny * nz, sys = nz;
    float **f = p.s0.f;
    float **ps = p.s0.psi;
    const float ex0 = f[FDTD_EX][c], ey0 = f[FDTD_EY][c], ez0 = f[FDTD_EZ][c];
    const float ex_y = (j + 1 < ny) ? f[FDTD_EX][c + sys] : 0.f;
    const float ex_z = (k + 1 < nz) ? f[FDTD_EX][c + 1] : 0.f;
    const float ey_x = (i + 1 < nx) ? f[FDTD_EY][c + sxs] : 0.f;
    const float ey_z = (k + 1 < nz) ? f[FDTD_EY][c + 1] : 0.f;
    const float ez_x = (i + 1 < nx) ? f[FDTD_EZ][c + sxs] : 0.f;
    const float ez_y = (j + 1 < ny) ? f[FDTD_EZ][c + sys] : 0.f;
    const float db = p.db ? p.db[c] : p.db0;
    const int ii = slab_index(p.x, i), jj = slab_index(p.y, j), kk = slab_index(p.z, k);
    const int sx = p.x.lo + p.x.hi, sy = p.y.lo + p.y.hi, sz = p.z.lo + p.z.hi;
    (void)sx;
    const float dEzy = ez_y - ez0, dEyz = ey_z - ey0;
    const float dExz = ex_z - ex0, dEzx = ez_x - ez0;
    const float dEyx = ey_x - ey0, dExy = ex_y - ex0;
    float a, b;
    // Hx
    a = p.y.kH[j] * dEzy;
    b = p.z.kH[k] * dEyz;
    if (jj >= 0) a += cpml_upd(ps[PSI_HXY], ps[PSI_HXY], ys_idx(i, jj, k, sy, nz), p.y.bH[j], p.y.cH[j], dEzy);
    if (kk >= 0) b += cpml_upd(ps[PSI_HXZ], ps[PSI_HXZ], zs_idx(i, j, kk, ny, sz), p.z.bH[k], p.z.cH[k], dEyz);
    f[FDTD_HX][c] -= db * (a - b);
    // Hy
    a = p.z.kH[k] * dExz;
    b = p.x.kH[i] * dEzx;
    if (kk >= 0) a += cpml_upd(ps[PSI_HYZ], ps[PSI_HYZ], zs_idx(i, j, kk, ny, sz), p.z.bH[k], p.z.cH[k], dExz);
    if (ii >= 0) b += cpml_upd(ps[PSI_HYX], ps[PSI_HYX], xs_idx(ii, j, k, ny, nz), p.x.bH[i], p.x.cH[i], dEzx);
    f[FDTD_HY][c] -= db * (a - b);
    // Hz
    a = p.x.kH[i] * dEyx;
    b = p.y.kH[j] * dExy;
    if (ii >= 0) a += cpml_upd(ps[PSI_HZX], ps[PSI_HZX], xs_idx(ii, j, k, ny, nz), p.x.bH[i], p.x.cH[i], dEyx);
    if (jj >= 0) b += cpml_upd(ps[PSI_HZY], ps[PSI_HZY], ys_idx(i, jj, k, sy, nz), p.y.bH[j], p.y.cH[j], dExy);
    f[FDTD_HZ][c] -= db * (a - b);
}

__global__ __launch_bounds__(256) void k3d_ref_e(Prob3D p, int64_t step) {
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int k = (int)(c % nz);
    const int j = (int)((c / nz) % ny);
    const int i = (int)(c / ((int64_t)ny * nz));
    const int64_t sxs = (int64_t)ny * nz, sys = nz;
    float **f = p.s0.f;
    float **ps = p.s0.psi;
    const int ii = slab_index(p.x, i), jj = slab_index(p.y, j), kk = slab_index(p.z, k);
    const int sy = p.y.lo + p.y.hi, sz = p.z.lo + p.z.hi;
    const float ca = p.ca ? p.ca[c] : 1.f;
    const float cb = p.cb[c];
    const float hx = f[FDTD_HX][c], hy = f[FDTD_HY][c], hz = f[FDTD_HZ][c];
    float a, b;
    if (j >= 1 && k >= 1) {
        const float dHzy = hz - f[FDTD_HZ][c - sys], dHyz = hy - f[FDTD_HY][c - 1];
        a = p.y.kE[j] * dHzy;
        b = p.z.kE[k] * dHyz;
        if (jj >= 0) a += cpml_upd(ps[PSI_EXY], ps[PSI_EXY], ys_idx(i, jj, k, sy, nz), p.y.bE[j], p.y.cE[j], dHzy);
        if (kk >= 0) b += cpml_upd(ps[PSI_EXZ], ps[PSI_EXZ], zs_idx(i, j, kk, ny, sz), p.z.bE[k], p.z.cE[k], dHyz);
        f[FDTD_EX][c] = ca * f[FDTD_EX][c] + cb * (a - b);
    }
    if (i >= 1 && k >= 1) {
        const float dHxz = hx - f[FDTD_HX][c - 1], dHzx = hz - f[FDTD_HZ][c - sxs];
        a = p.z.kE[k] * dHxz;
        b = p.x.kE[i] * dHzx;
        if (kk >= 0) a += cpml_upd(ps[PSI_EYZ], ps[PSI_EYZ], zs_idx(i, j, kk, ny, sz), p.z.bE[k], p.z.cE[k], dHxz);
        if (ii >= 0) b += cpml_upd(ps[PSI_EYX], ps[PSI_EYX], xs_idx(ii, j, k, ny, nz), p.x.bE[i], p.x.cE[i], dHzx);
        f[FDTD_EY][c] = ca * f[FDTD_EY][c] + cb * (a - b);
    }
    if (i >= 1 && j >= 1) {
        const float dHyx = hy - f[FDTD_HY][c - sxs], dHxy = hx - f[FDTD_HX][c - sys];
        a = p.x.kE[i] * dHyx;
        b = p.y.kE[j] * dHxy;
        if (ii >= 0) a += cpml_upd(ps[PSI_EZX], ps[PSI_EZX], xs_idx(ii, j, k, ny, nz), p.x.bE[i], p.x.cE[i], dHyx);
        if (jj >= 0) b += cpml_upd(ps[PSI_EZY], ps[PSI_EZY], ys_idx(i, jj, k, sy, nz), p.y.bE[j], p.y.cE[j], dHxy);
        f[FDTD_EZ][c] = ca * f[FDTD_EZ][c] + cb * (a - b);
    }
    if (c == p.src_idx && step < p.src_len) f[p.src_comp][c] += p.src_vals[step];
}

__global__ void k_probe_3d(Prob3D p, int64_t step) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < p.np)
        p.rec[(int64_t)q * p.rec_stride + (step - p.rec_base)] = p.s0.f[p.probe_comp][p.probe_idx[q]];
}

hipError_t launch_3d_ref(const Prob3D &p, int64_t step, hipStream_t st) {
    const int64_t n = (int64_t)p.nx * p.ny * p.nz;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k3d_ref_h, dim3(nb), dim3(256), 0, st, p);
    hipLaunchKernelGGL(k3d_ref_e, dim3(nb), dim3(256), 0, st, p, step);
    if (p.np > 0)
        hipLaunchKernelGGL(k_probe_3d, dim3((p.np + 63) / 64), dim3(64), 0, st, p, step);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused single pass (2.5D).
//
// A workgroup owns TJ consecutive y rows times the whole z line of a chunk of
// TX x planes, and marches along x.  Thread t holds z = t + m*BZ (m < M) of
// all its rows in registers, together with the E plane i, the E plane i+1
// and the H plane i-1.  y neighbours are in the thread's own registers (the
// rows j0-1 and j0+TJ are loaded as halo, and H of row j0-1 is recomputed);
// z neighbours go through LDS; x neighbours are the carried planes (the H
// plane x0-1 is recomputed at the start).  State is double buffered
// (read s0, write s1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_block3(int b, int nb) {
    return (nb % 8 == 0) ? (b % 8) * (nb / 8) + (b / 8) : b;
}

template <int TJ, int M, bool PML>
__global__ __launch_bounds__(256) void k3d_fused(Prob3D p, int TX, int njt, int ntiles,
                                                 ProbeTiles pt, int64_t step) {
    extern __shared__ float lds[];
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int BZ = blockDim.x;
    const int NZP = BZ * M;
    float *lEy = lds;                        // rows -1..TJ-1
    float *lEx = lEy + (TJ + 1) * NZP;       // rows 0..TJ-1
    float *lHy = lEx + TJ * NZP;             // rows 0..TJ-1
    float *lHx = lHy + TJ * NZP;             // rows 0..TJ-1

    const int t = xcd_block3(blockIdx.x, gridDim.x);
    if (t >= ntiles) return;  // uniform over the block
    const int cx = t / njt, jt = t - cx * njt;
    const int x0 = cx * TX, x1 = min(x0 + TX, nx);
    const int j0 = jt * TJ;
    const int64_t PL = (int64_t)ny * nz;  // plane stride
    const bool lossy = p.ca != nullptr, mumap = p.db != nullptr;
    const int sy = p.y.lo + p.y.hi, sz = p.z.lo + p.z.hi;

    int kq[M];
    bool kv[M];
    float kHz[M], kEz[M], bHz[M], cHz[M], bEz[M], cEz[M];
    int kk[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        kq[m] = threadIdx.x + m * BZ;
        kv[m] = kq[m] < nz;
        const int k = kv[m] ? kq[m] : 0;
        kHz[m] = p.z.kH[k];
        kEz[m] = p.z.kE[k];
        kk[m] = -1;
        bHz[m] = cHz[m] = bEz[m] = cEz[m] = 0.f;
        if (PML && kv[m]) {
            kk[m] = slab_index(p.z, k);
            if (kk[m] >= 0) {
                bHz[m] = p.z.bH[k]; cHz[m] = p.z.cH[k];
                bEz[m] = p.z.bE[k]; cEz[m] = p.z.cE[k];
            }
        }
    }
    // row validity and y profiles (rows -1..TJ, index r+1)
    bool rv[TJ + 2];
    float kHy[TJ + 1], kEy[TJ + 1];
    int jjr[TJ + 1];
#pragma unroll
    for (int r = -1; r <= TJ; ++r) {
        const int j = j0 + r;
        rv[r + 1] = (j >= 0 && j < ny);
        if (r < TJ) {
            const int jc = rv[r + 1] ? j : 0;
            kHy[r + 1] = p.y.kH[jc];
            kEy[r + 1] = p.y.kE[jc];
            jjr[r + 1] = (PML && rv[r + 1]) ? slab_index(p.y, jc) : -1;
        }
    }

    float ex_c[TJ + 2][M], ey_c[TJ + 2][M], ez_c[TJ + 2][M];
    float hy_p[TJ][M], hz_p[TJ][M];
    const int istart = (x0 > 0) ? x0 - 1 : x0;
    // load E plane istart
#pragma unroll
    for (int r = -1; r <= TJ; ++r)
#pragma unroll
        for (int m = 0; m < M; ++m) {
            ex_c[r + 1][m] = ey_c[r + 1][m] = ez_c[r + 1][m] = 0.f;
            if (rv[r + 1] && kv[m]) {
                const int64_t c = istart * PL + (int64_t)(j0 + r) * nz + kq[m];
                ex_c[r + 1][m] = p.s0.f[FDTD_EX][c];
                if (r < TJ) ey_c[r + 1][m] = p.s0.f[FDTD_EY][c];
                ez_c[r + 1][m] = p.s0.f[FDTD_EZ][c];
            }
        }
#pragma unroll
    for (int r = 0; r < TJ; ++r)
#pragma unroll
        for (int m = 0; m < M; ++m) hy_p[r][m] = hz_p[r][m] = 0.f;

    const int pbeg = pt.start[t], pend = pt.start[t + 1];
    const float sval = (p.src_idx >= 0 && step < p.src_len) ? p.src_vals[step] : 0.f;

    for (int i = istart; i < x1; ++i) {
        const bool own = i >= x0;
        const int64_t pb = (int64_t)i * PL;
        // ---- loads: E plane i+1, H plane i, coefficients ----
        float ex_n[TJ + 2][M], ey_n[TJ + 2][M], ez_n[TJ + 2][M];
        float hx_o[TJ + 1][M], hy_o[TJ][M], hz_o[TJ + 1][M], db[TJ + 1][M];
        float cb[TJ][M], ca[TJ][M];
#pragma unroll
        for (int r = -1; r <= TJ; ++r)
#pragma unroll
            for (int m = 0; m < M; ++m) {
                ex_n[r + 1][m] = ey_n[r + 1][m] = ez_n[r + 1][m] = 0.f;
                const bool ok = rv[r + 1] && kv[m];
                const int64_t c = pb + (int64_t)(j0 + r) * nz + kq[m];
                if (ok && i + 1 < nx) {
                    ex_n[r + 1][m] = p.s0.f[FDTD_EX][c + PL];
                    if (r < TJ) ey_n[r + 1][m] = p.s0.f[FDTD_EY][c + PL];
                    ez_n[r + 1][m] = p.s0.f[FDTD_EZ][c + PL];
                }
                if (r < TJ) {
                    hx_o[r + 1][m] = hz_o[r + 1][m] = 0.f;
                    db[r + 1][m] = p.db0;
                    if (ok) {
                        hx_o[r + 1][m] = p.s0.f[FDTD_HX][c];
                        hz_o[r + 1][m] = p.s0.f[FDTD_HZ][c];
                        if (mumap) db[r + 1][m] = p.db[c];
                    }
                    if (r >= 0) {
                        hy_o[r][m] = 0.f;
                        cb[r][m] = 0.f;
                        ca[r][m] = 1.f;
                        if (ok) {
                            hy_o[r][m] = p.s0.f[FDTD_HY][c];
                            if (own) {
                                cb[r][m] = p.cb[c];
                                if (lossy) ca[r][m] = p.ca[c];
                            }
                        }
                    }
                }
            }
        // ---- E plane i to LDS (z neighbours for the H layer) ----
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int k = kq[m];
#pragma unroll
            for (int r = -1; r < TJ; ++r) lEy[(r + 1) * NZP + k] = ey_c[r + 1][m];
#pragma unroll
            for (int r = 0; r < TJ; ++r) lEx[r * NZP + k] = ex_c[r + 1][m];
        }
        __syncthreads();
        // ---- H layer, plane i ----
        const float kHx = p.x.kH[i];
        const int ii = PML ? slab_index(p.x, i) : -1;
        float hx_n[TJ + 1][M], hy_n[TJ][M], hz_n[TJ + 1][M];
#pragma unroll
        for (int r = -1; r < TJ; ++r) {
            const int j = j0 + r;
            const int jj = jjr[r + 1];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int k = kq[m];
                const bool ok = rv[r + 1] && kv[m];
                const bool wr = ok && own && r >= 0;
                const float eyz1 = (k + 1 < nz) ? lEy[(r + 1) * NZP + k + 1] : 0.f;
                // Hx
                const float dEzy = ez_c[r + 2][m] - ez_c[r + 1][m];
                const float dEyz = eyz1 - ey_c[r + 1][m];
                float a = kHy[r + 1] * dEzy, b = kHz[m] * dEyz;
                if (PML && ok) {
                    if (jj >= 0) {
                        const int64_t q = ys_idx(i, jj, k, sy, nz);
                        const float ps = p.y.bH[j] * p.s0.psi[PSI_HXY][q] + p.y.cH[j] * dEzy;
                        if (wr) p.s1.psi[PSI_HXY][q] = ps;
                        a += ps;
                    }
                    if (kk[m] >= 0) {
                        const int64_t q = zs_idx(i, j, kk[m], ny, sz);
                        const float ps = bHz[m] * p.s0.psi[PSI_HXZ][q] + cHz[m] * dEyz;
                        if (wr) p.s1.psi[PSI_HXZ][q] = ps;
                        b += ps;
                    }
                }
                hx_n[r + 1][m] = hx_o[r + 1][m] - db[r + 1][m] * (a - b);
                // Hz
                const float dEyx = ey_n[r + 1][m] - ey_c[r + 1][m];
                const float dExy = ex_c[r + 2][m] - ex_c[r + 1][m];
                a = kHx * dEyx;
                b = kHy[r + 1] * dExy;
                if (PML && ok) {
                    if (ii >= 0) {
                        const int64_t q = xs_idx(ii, j, k, ny, nz);
                        const float ps = p.x.bH[i] * p.s0.psi[PSI_HZX][q] + p.x.cH[i] * dEyx;
                        if (wr) p.s1.psi[PSI_HZX][q] = ps;
                        a += ps;
                    }
                    if (jj >= 0) {
                        const int64_t q = ys_idx(i, jj, k, sy, nz);
                        const float ps = p.y.bH[j] * p.s0.psi[PSI_HZY][q] + p.y.cH[j] * dExy;
                        if (wr) p.s1.psi[PSI_HZY][q] = ps;
                        b += ps;
                    }
                }
                hz_n[r + 1][m] = hz_o[r + 1][m] - db[r + 1][m] * (a - b);
                // Hy (own rows only)
                if (r >= 0) {
                    const float exz1 = (k + 1 < nz) ? lEx[r * NZP + k + 1] : 0.f;
                    const float dExz = exz1 - ex_c[r + 1][m];
                    const float dEzx = ez_n[r + 1][m] - ez_c[r + 1][m];
                    a = kHz[m] * dExz;
                    b = kHx * dEzx;
                    if (PML && ok) {
                        if (kk[m] >= 0) {
                            const int64_t q = zs_idx(i, j, kk[m], ny, sz);
                            const float ps = bHz[m] * p.s0.psi[PSI_HYZ][q] + cHz[m] * dExz;
                            if (wr) p.s1.psi[PSI_HYZ][q] = ps;
                            a += ps;
                        }
                        if (ii >= 0) {
                            const int64_t q = xs_idx(ii, j, k, ny, nz);
                            const float ps = p.x.bH[i] * p.s0.psi[PSI_HYX][q] + p.x.cH[i] * dEzx;
                            if (wr) p.s1.psi[PSI_HYX][q] = ps;
                            b += ps;
                        }
                    }
                    hy_n[r][m] = hy_o[r][m] - db[r + 1][m] * (a - b);
                }
            }
        }
        // ---- H plane i to LDS (z neighbours for the E layer) ----
#pragma unroll
        for (int m = 0; m < M; ++m)
#pragma unroll
            for (int r = 0; r < TJ; ++r) {
                lHy[r * NZP + kq[m]] = hy_n[r][m];
                lHx[r * NZP + kq[m]] = hx_n[r + 1][m];
            }
        __syncthreads();
        if (own) {
            const float kEx = p.x.kE[i];
            float ex_w[TJ][M], ey_w[TJ][M], ez_w[TJ][M];
#pragma unroll
            for (int r = 0; r < TJ; ++r) {
                const int j = j0 + r;
                const int jj = jjr[r + 1];
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const int k = kq[m];
                    const bool ok = rv[r + 1] && kv[m];
                    const int64_t c = pb + (int64_t)j * nz + k;
                    ex_w[r][m] = ex_c[r + 1][m];
                    ey_w[r][m] = ey_c[r + 1][m];
                    ez_w[r][m] = ez_c[r + 1][m];
                    const float hyz0 = (k >= 1) ? lHy[r * NZP + k - 1] : 0.f;
                    const float hxz0 = (k >= 1) ? lHx[r * NZP + k - 1] : 0.f;
                    float a, b;
                    if (ok && j >= 1 && k >= 1) {  // Ex
                        const float dHzy = hz_n[r + 1][m] - hz_n[r][m];
                        const float dHyz = hy_n[r][m] - hyz0;
                        a = kEy[r + 1] * dHzy;
                        b = kEz[m] * dHyz;
                        if (PML) {
                            if (jj >= 0) a += cpml_upd(p.s0.psi[PSI_EXY], p.s1.psi[PSI_EXY], ys_idx(i, jj, k, sy, nz), p.y.bE[j], p.y.cE[j], dHzy);
                            if (kk[m] >= 0) b += cpml_upd(p.s0.psi[PSI_EXZ], p.s1.psi[PSI_EXZ], zs_idx(i, j, kk[m], ny, sz), bEz[m], cEz[m], dHyz);
                        }
                        ex_w[r][m] = (lossy ? ca[r][m] * ex_c[r + 1][m] : ex_c[r + 1][m]) + cb[r][m] * (a - b);
                    }
                    if (ok && i >= 1 && k >= 1) {  // Ey
                        const float dHxz = hx_n[r + 1][m] - hxz0;
                        const float dHzx = hz_n[r + 1][m] - hz_p[r][m];
                        a = kEz[m] * dHxz;
                        b = kEx * dHzx;
                        if (PML) {
                            if (kk[m] >= 0) a += cpml_upd(p.s0.psi[PSI_EYZ], p.s1.psi[PSI_EYZ], zs_idx(i, j, kk[m], ny, sz), bEz[m], cEz[m], dHxz);
                            if (ii >= 0) b += cpml_upd(p.s0.psi[PSI_EYX], p.s1.psi[PSI_EYX], xs_idx(ii, j, k, ny, nz), p.x.bE[i], p.x.cE[i], dHzx);
                        }
                        ey_w[r][m] = (lossy ? ca[r][m] * ey_c[r + 1][m] : ey_c[r + 1][m]) + cb[r][m] * (a - b);
                    }
                    if (ok && i >= 1 && j >= 1) {  // Ez
                        const float dHyx = hy_n[r][m] - hy_p[r][m];
                        const float dHxy = hx_n[r + 1][m] - hx_n[r][m];
                        a = kEx * dHyx;
                        b = kEy[r + 1] * dHxy;
                        if (PML) {
                            if (ii >= 0) a += cpml_upd(p.s0.psi[PSI_EZX], p.s1.psi[PSI_EZX], xs_idx(ii, j, k, ny, nz), p.x.bE[i], p.x.cE[i], dHyx);
                            if (jj >= 0) b += cpml_upd(p.s0.psi[PSI_EZY], p.s1.psi[PSI_EZY], ys_idx(i, jj, k, sy, nz), p.y.bE[j], p.y.cE[j], dHxy);
                        }
                        ez_w[r][m] = (lossy ? ca[r][m] * ez_c[r + 1][m] : ez_c[r + 1][m]) + cb[r][m] * (a - b);
                    }
                    if (c == p.src_idx) {
                        if (p.src_comp == FDTD_EX) ex_w[r][m] += sval;
                        else if (p.src_comp == FDTD_EY) ey_w[r][m] += sval;
                        else ez_w[r][m] += sval;
                    }
                    if (ok) {
                        p.s1.f[FDTD_EX][c] = ex_w[r][m];
                        p.s1.f[FDTD_EY][c] = ey_w[r][m];
                        p.s1.f[FDTD_EZ][c] = ez_w[r][m];
                        p.s1.f[FDTD_HX][c] = hx_n[r + 1][m];
                        p.s1.f[FDTD_HY][c] = hy_n[r][m];
                        p.s1.f[FDTD_HZ][c] = hz_n[r + 1][m];
                    }
                }
            }
            // probes of this tile in plane i
            for (int q = pbeg; q < pend; ++q) {
                const int64_t cell = pt.cell[q];
                const int pi = (int)(cell / PL);
                if (pi != i) continue;
                const int pj = (int)((cell / nz) % ny);
                const int pk = (int)(cell % nz);
#pragma unroll
                for (int r = 0; r < TJ; ++r)
#pragma unroll
                    for (int m = 0; m < M; ++m)
                        if (pj == j0 + r && pk == kq[m]) {
                            float v;
                            switch (p.probe_comp) {
                                case FDTD_EX: v = ex_w[r][m]; break;
                                case FDTD_EY: v = ey_w[r][m]; break;
                                case FDTD_EZ: v = ez_w[r][m]; break;
                                case FDTD_HX: v = hx_n[r + 1][m]; break;
                                case FDTD_HY: v = hy_n[r][m]; break;
                                default: v = hz_n[r + 1][m]; break;
                            }
                            p.rec[(int64_t)pt.slot[q] * p.rec_stride + (step - p.rec_base)] = v;
                        }
            }
        }
        // carry
#pragma unroll
        for (int r = 0; r < TJ; ++r)
#pragma unroll
            for (int m = 0; m < M; ++m) {
                hy_p[r][m] = hy_n[r][m];
                hz_p[r][m] = hz_n[r + 1][m];
            }
#pragma unroll
        for (int r = 0; r < TJ + 2; ++r)
#pragma unroll
            for (int m = 0; m < M; ++m) {
                ex_c[r][m] = ex_n[r][m];
                ey_c[r][m] = ey_n[r][m];
                ez_c[r][m] = ez_n[r][m];
            }
    }
}

static int bz_of(int nz) {
    int bz = ((nz + 63) / 64) * 64;
    if (bz > 256) bz = 256;
    return bz;
}

int fused3d_ntiles(int nx, int ny, int nz, const Fused3DCfg &c) {
    (void)nz;
    return ((nx + c.TX - 1) / c.TX) * ((ny + c.TJ - 1) / c.TJ);
}

int fused3d_tile_of(int nx, int ny, int nz, const Fused3DCfg &c, int i, int j, int k) {
    (void)nx; (void)nz; (void)k;
    const int njt = (ny + c.TJ - 1) / c.TJ;
    return (i / c.TX) * njt + j / c.TJ;
}

bool fused3d_supported(int nx, int ny, int nz, const Fused3DCfg &c) {
    (void)nx; (void)ny;
    const int bz = bz_of(nz);
    const int M = (nz + bz - 1) / bz;
    if (!(c.TJ == 1 || c.TJ == 2 || c.TJ == 4 || c.TJ == 8)) return false;
    if (!(M == 1 || M == 2 || M == 4)) return false;
    const size_t lds = (size_t)(4 * c.TJ + 1) * bz * M * sizeof(float);
    return c.TX >= 1 && lds <= 160 * 1024;
}

template <int TJ, int M, bool PML>
static void go3d(const Prob3D &p, const Fused3DCfg &c, const ProbeTiles &pt, int64_t step,
                 hipStream_t st, int bz) {
    const int njt = (p.ny + TJ - 1) / TJ;
    const int ntiles = fused3d_ntiles(p.nx, p.ny, p.nz, c);
    const size_t lds = (size_t)(4 * TJ + 1) * bz * M * sizeof(float);
    hipLaunchKernelGGL((k3d_fused<TJ, M, PML>), dim3(ntiles), dim3(bz), lds, st, p, c.TX, njt,
                       ntiles, pt, step);
}

hipError_t launch_3d_fused(const Prob3D &p, const Fused3DCfg &c, const ProbeTiles &pt,
                           int64_t step, hipStream_t st) {
    if (!fused3d_supported(p.nx, p.ny, p.nz, c)) return hipErrorInvalidValue;
    const bool pml = (p.x.lo + p.x.hi + p.y.lo + p.y.hi + p.z.lo + p.z.hi) > 0;
    const int bz = bz_of(p.nz);
    const int M = (p.nz + bz - 1) / bz;
#define GEM_GO3(TJ_, M_)                                         \
    do {                                                         \
        if (pml) go3d<TJ_, M_, true>(p, c, pt, step, st, bz);    \
        else go3d<TJ_, M_, false>(p, c, pt, step, st, bz);       \
    } while (0)
#define GEM_GO3M(TJ_)                     \
    do {                                  \
        if (M == 1) GEM_GO3(TJ_, 1);      \
        else if (M == 2) GEM_GO3(TJ_, 2); \
        else GEM_GO3(TJ_, 4);             \
    } while (0)
    switch (c.TJ) {
        case 1: GEM_GO3M(1); break;
        case 2: GEM_GO3M(2); break;
        case 4: GEM_GO3M(4); break;
        case 8: GEM_GO3M(8); break;
        default: return hipErrorInvalidValue;
    }
#undef GEM_GO3M
#undef GEM_GO3
    return hipGetLastError();
}

}  // namespace gem
