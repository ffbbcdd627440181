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
    if (p.src_idx >= 0 && in_src(p.src_box, i, j, k) && step < p.src_len) f[p.src_comp][c] += p.src_vals[step];
}

__global__ void k_probe_3d(Prob3D p, int64_t step) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < p.np)
        p.rec[(int64_t)q * p.rec_stride + (step - p.rec_base)] = p.s0.f[p.probe_comp][p.probe_idx[q]];
}

// probe q of a list: rec[slot[q]][step] = component of set s0 at cell[q]
__global__ void k_probe_3d_list(Prob3D p, const int *cell, const int *slot, int n, int64_t step) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) p.rec[(int64_t)slot[q] * p.rec_stride + (step - p.rec_base)] = p.s0.f[p.probe_comp][cell[q]];
}

hipError_t launch_3d_probe_list(const Prob3D &p, const int *cell, const int *slot, int n, int64_t step,
                                hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_3d_list, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, p, cell, slot, n, step);
    return hipGetLastError();
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

}  // namespace gem
