// Device copy of the STREAM "copy" kind: the practical ceiling of the HBM
// bandwidth that every kernel of the library is compared with.  One 16-byte
// vector per thread, one thread per vector (no grid-stride loop): on 1-4 GiB
// buffers this form moved the most bytes per second of the copy kernels
// tried (grid-stride loops of 1-8 vectors per thread, non-temporal loads and
// stores).
#include <hip/hip_runtime.h>

#include <string>

#include "sim.hpp"

namespace gem {

int status_of_current_exception();

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_stream_copy(const v4f *__restrict__ a, v4f *__restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}

}  // namespace

}  // namespace gem

using namespace gem;

extern "C" int fdtd_stream_copy(void *dst, const void *src, size_t bytes, void *stream) {
    try {
        if (!dst || !src) fail(FDTD_EINVAL, "NULL argument");
        if (bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0)
            fail(FDTD_EINVAL, "bytes and both addresses must be multiples of 16");
        const int64_t n = (int64_t)(bytes / 16);
        if (n == 0) return FDTD_OK;
        const int64_t blocks = (n + 255) / 256;
        if (blocks > INT32_MAX) fail(FDTD_EINVAL, "copy too large");
        hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                           (const v4f *)src, (v4f *)dst, n);
        hip_check(hipGetLastError(), "stream copy");
        return FDTD_OK;
    } catch (...) {
        return status_of_current_exception();
    }
}
