// Frequency-domain monitor: running discrete Fourier transform of one field
// component at a list of cells, fed after every step (the paper motivates
// frequency-domain responses, Sec. I, without a formulation).  One thread per
// cell; the step's phase factors arrive by value, so the kernel reads the
// field once and updates its FP64 sums.
#include "common.hpp"

namespace gem {

__global__ __launch_bounds__(256) void k_dft(const float *__restrict__ f, const int64_t *__restrict__ idx,
                                             int64_t npts, int nf, DftPhase ph, double *__restrict__ acc) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= npts) return;
    const double v = f[idx[c]];
    for (int q = 0; q < nf; ++q) {
        acc[(2 * q) * npts + c] += v * ph.re[q];
        acc[(2 * q + 1) * npts + c] += v * ph.im[q];
    }
}

hipError_t launch_dft(const float *f, const int64_t *idx, int64_t npts, int nf, const DftPhase &ph, double *acc,
                      hipStream_t st) {
    if (npts <= 0) return hipSuccess;
    if (nf < 1 || nf > kDftMaxFreq) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dft, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, f, idx, npts, nf, ph, acc);
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
