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

}  // namespace gem
