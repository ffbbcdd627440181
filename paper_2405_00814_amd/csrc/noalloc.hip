// Probe read-out that allocates no device memory.
//
// fdtd_probe gathers the probe rows (stored with a row stride of the record
// capacity) into one packed block of device memory and copies that block to
// the host.  fdtd_probe_noalloc does the same through `scratch`, a fixed
// device array of this file, so that callers which must not allocate (code
// that runs while a HIP graph is being captured on other streams, serving
// loops, harnesses that forbid allocation) can still read the records.
//
// Each device that runs the library holds its own copy of `scratch` until
// the process ends.  Its device address is looked up once per device (with
// that device current) on the first call there and kept; host code never
// passes the array's name to a kernel.  Every call on one device uses the
// same array: calls that overlap on one device (different threads or
// streams) race.  The gather writes every entry it later copies, so nothing
// has to be cleared between calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "sim.hpp"

namespace gem {

int status_of_current_exception();

constexpr int64_t kScratchFloats = (int64_t)4 << 20;  // 16 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) float scratch[kScratchFloats];

namespace {

std::mutex g_mtx;
float *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (looked up once, with the device
// current).
float *scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) fail(FDTD_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mtx);
    if (g_ptr[device]) return g_ptr[device];
    int prev = -1;
    hip_check(hipGetDevice(&prev), "hipGetDevice");
    if (prev != device) hip_check(hipSetDevice(device), "hipSetDevice");
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    hip_check(e, "hipGetSymbolAddress(scratch)");
    if (!p) fail(FDTD_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_ptr[device] = (float *)p;
    return g_ptr[device];
}

// out[p * m + s] = rec[p * stride + s] for p < np, s < m.
__global__ void k_pack_records(const float *__restrict__ rec, int64_t stride, int64_t m, int64_t np,
                               float *__restrict__ out) {
    const int64_t total = np * m;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = q / m, s = q - p * m;
        out[q] = rec[p * stride + s];
    }
}

}  // namespace

}  // namespace gem

using namespace gem;

extern "C" int fdtd_probe_noalloc(fdtd_sim *sim, float *out, int64_t cap, int64_t *n_recorded) {
    try {
        if (!sim) fail(FDTD_EINVAL, "sim is NULL");
        Sim &s = sim->s;
        if (n_recorded) *n_recorded = s.n_rec;
        if (!out || s.probe_cells.empty()) return FDTD_OK;
        if (cap < 0) fail(FDTD_EINVAL, "cap must be >= 0");
        const int64_t P = (int64_t)s.probe_cells.size();
        const int64_t m = std::min(cap, s.n_rec);
        if (m == 0) return FDTD_OK;
        if (P * m > kScratchFloats)
            fail(FDTD_EINVAL, "probes x samples = " + std::to_string(P * m) +
                                  " floats exceeds the no-allocation limit of " + std::to_string(kScratchFloats) +
                                  " floats (16 MiB); read fewer samples per call or use fdtd_probe");
        float *buf = scratch_ptr(s.device);
        const int64_t total = P * m;
        const int threads = 256;
        const int64_t want = (total + threads - 1) / threads;
        const int blocks = (int)std::min<int64_t>(want, 4096);
        hipLaunchKernelGGL(k_pack_records, dim3(blocks), dim3(threads), 0, s.st, s.rec_dev, s.rec_cap, m, P, buf);
        hip_check(hipGetLastError(), "record pack");
        if (cap == m) {
            hip_check(hipMemcpyAsync(out, buf, (size_t)total * sizeof(float), hipMemcpyDeviceToHost, s.st),
                      "record copy");
        } else {
            for (int64_t p = 0; p < P; ++p)
                hip_check(hipMemcpyAsync(out + p * cap, buf + p * m, (size_t)m * sizeof(float),
                                         hipMemcpyDeviceToHost, s.st),
                          "record copy");
        }
        hip_check(hipStreamSynchronize(s.st), "sync");
        return FDTD_OK;
    } catch (...) {
        return status_of_current_exception();
    }
}
