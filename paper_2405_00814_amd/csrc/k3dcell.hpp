// Device helpers shared by the 3D kernels (not included by host code).
#pragma once

#include "common.hpp"
#include "devutil.hpp"

namespace gem {

// linear index into the x-, y- and z-slab psi arrays
__device__ __forceinline__ unsigned xs3(int ii, int j, int k, int ny, int nz) {
    return ((unsigned)ii * ny + j) * nz + k;
}
__device__ __forceinline__ unsigned ys3(int i, int jj, int k, int sy, int nz) {
    return ((unsigned)i * sy + jj) * nz + k;
}
__device__ __forceinline__ unsigned zs3(int i, int j, int kk, int ny, int sz) {
    return ((unsigned)i * ny + j) * sz + kk;
}

// Profile of one axis at one index (b, c of the CPML recursion; 1/(kappa d)).
// For x and y the index is uniform over a wavefront, so these are scalar loads.
struct AxP {
    float kH, kE, bH, cH, bE, cE;
    int s;  // slab index or -1
};
template <bool PML>
__device__ __forceinline__ AxP axp(const AxisDev &a, int i) {
    AxP r;
    r.kH = a.kH[i];
    r.kE = a.kE[i];
    r.s = PML ? slab_index(a, i) : -1;
    r.bH = r.cH = r.bE = r.cE = 0.f;
    if (PML && r.s >= 0) {
        r.bH = a.bH[i]; r.cH = a.cH[i];
        r.bE = a.bE[i]; r.cE = a.cE[i];
    }
    return r;
}

// value at z+1 of element q of a lane's vector: the next element, or the
// next lane's first element, or (the segment's last lane) the seam value
template <int V>
__device__ __forceinline__ float znext(const float (&x)[V], int q, float seam, bool last) {
    if (q + 1 < V) return x[q + 1];
    const float s = lane_next(x[0]);
    return last ? seam : s;
}

}  // namespace gem
