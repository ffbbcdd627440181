// Frequency-domain monitor: running discrete Fourier transform of one field
// component at a box of cells, fed after every step (the paper motivates
// frequency-domain responses, Sec. I, without a formulation).  The FP64 sums
// cost 16 B of reads and writes per frequency and update, so the samples of
// kDftBatch steps are first gathered into a ring (8 B per cell and step:
// one read, one write) and the sums updated once per batch with the
// buffered steps' phase factors, passed by value: per cell and step about
// 4 + 32 nf / kDftBatch bytes instead of 4 + 32 nf.  One thread per cell.
#include "common.hpp"

namespace gem {

__global__ __launch_bounds__(256) void k_dft_gather(const float *__restrict__ f, const int64_t *__restrict__ idx,
                                                    DftBox b, int64_t npts, float *__restrict__ row) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= npts) return;
    int64_t g;
    if (idx) {
        g = idx[c];
    } else {
        const int64_t k = c % b.nk, r = c / b.nk;
        const int64_t j = r % b.nj, i = r / b.nj;
        g = ((b.i0 + i) * b.ny + (b.j0 + j)) * b.nz + (b.k0 + k);
    }
    row[c] = f[g];
}

__global__ __launch_bounds__(256) void k_dft_flush(const float *__restrict__ ring, int64_t npts, int nk, int nf,
                                                   DftPhases ph, double *__restrict__ acc) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= npts) return;
    double v[kDftBatch];
#pragma unroll
    for (int k = 0; k < kDftBatch; ++k) v[k] = k < nk ? (double)ring[k * npts + c] : 0.0;
    for (int q = 0; q < nf; ++q) {
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int k = 0; k < kDftBatch; ++k) {
            re += v[k] * ph.re[k][q];
            im += v[k] * ph.im[k][q];
        }
        acc[(2 * q) * npts + c] += re;
        acc[(2 * q + 1) * npts + c] += im;
    }
}

hipError_t launch_dft_gather(const float *f, const int64_t *idx, const DftBox &box, int64_t npts, float *row,
                             hipStream_t st) {
    if (npts <= 0) return hipSuccess;
    if (!idx && (box.nj < 1 || box.nk < 1)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dft_gather, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, f, idx, box, npts, row);
    return hipGetLastError();
}

hipError_t launch_dft_flush(const float *ring, int64_t npts, int nk, int nf, const DftPhases &ph, double *acc,
                            hipStream_t st) {
    if (npts <= 0 || nk == 0) return hipSuccess;
    if (nf < 1 || nf > kDftMaxFreq || nk < 0 || nk > kDftBatch) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dft_flush, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, ring, npts, nk, nf, ph,
                       acc);
    return hipGetLastError();
}

// The monitored E component's share of the specific absorption rate: the
// time-averaged power a time-harmonic field of complex amplitude X deposits
// per unit mass is sigma |X|^2 / (2 rho).  One thread per cell, all
// frequencies.
__global__ __launch_bounds__(256) void k_sar(const double *__restrict__ acc, int64_t npts, int nf,
                                             const float *__restrict__ sig, const float *__restrict__ rho,
                                             SarScale sc, float *__restrict__ out) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= npts) return;
    const double w = (double)sig[c] / (double)rho[c];
    for (int q = 0; q < nf; ++q) {
        const double re = acc[(2 * q) * npts + c], im = acc[(2 * q + 1) * npts + c];
        out[(int64_t)q * npts + c] = (float)(w * (re * re + im * im) * sc.inv2n2[q]);
    }
}

hipError_t launch_sar(const double *acc, int64_t npts, int nf, const float *sig, const float *rho,
                      const SarScale &sc, float *out, hipStream_t st) {
    if (npts <= 0) return hipSuccess;
    if (nf < 1 || nf > kDftMaxFreq) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sar, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, acc, npts, nf, sig, rho, sc,
                       out);
    return hipGetLastError();
}

}  // namespace gem
