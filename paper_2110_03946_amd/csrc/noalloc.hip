// Allocation-free variant of the one-sweep entry point (ddi_oras_sweep):
// the device scratch it needs -- the column-transposed mask bits, the
// per-block float64 norm partials and their per-channel sums -- lives in a
// fixed array of device memory that the library holds for the lifetime of
// the process, one copy per GPU, instead of being allocated per call. For
// callers that cannot call hipMalloc (code under graph capture, serving
// loops that forbid allocation). Host code only apart from the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "plan.h"

using namespace ddi;

namespace {

// The scratch array. Its name is a host-side stand-in in host code: every
// host use goes through the device address hipGetSymbolAddress returns for
// the current device (scratch_ptr).
static __device__ __align__(256) unsigned char scratch[DDI_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of the scratch array, looked up once
// per device with that device current.
int scratch_ptr(void** out) {
    int dev = 0;
    DDI_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return DDI_ENODEV;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        DDI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return DDI_EHIP;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return DDI_OK;
}

size_t round256(size_t n) { return (n + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

int ddi_noalloc_scratch_bytes(int height, int width, int channels, int block, int overlap_px,
                              size_t* bytes) {
    if (!bytes) return DDI_EINVAL;
    int e = check_dims(height, width, channels);
    if (e) return e;
    if (block < 2 || block > DDI_MAX_BLOCK || overlap_px < 0 || overlap_px >= block)
        return DDI_EINVAL;
    const SweepArgs a = make_sweep(height, width, channels, block, overlap_px, 1.f, 1);
    *bytes = round256((size_t)mask_bit_groups(height) * width * sizeof(uint64_t)) +
             round256((size_t)sweep_partials(a) * channels * sizeof(double)) +
             round256((size_t)channels * sizeof(double));
    return DDI_OK;
}

int ddi_oras_sweep_noalloc(const float* u_in, const uint8_t* c, float* u_out, int height,
                           int width, int channels, int block, int overlap_px,
                           float robin_alpha, int local_iters, double* rsq, void* stream) {
    size_t need = 0;
    int e = ddi_noalloc_scratch_bytes(height, width, channels, block, overlap_px, &need);
    if (e) return e;
    if (!u_in || !c || !u_out) return DDI_EINVAL;
    if (!(robin_alpha > 0.f && robin_alpha <= 1.f) || local_iters < 1) return DDI_EINVAL;
    const size_t nimg = (size_t)channels * height * width * sizeof(float);
    if (overlaps(u_out, nimg, u_in, nimg) || overlaps(u_out, nimg, c, (size_t)height * width))
        return DDI_EINVAL;
    if (need > (size_t)DDI_NOALLOC_SCRATCH_BYTES) return DDI_ESCRATCH;
    if ((e = check_device())) return e;
    void* base = nullptr;
    if ((e = scratch_ptr(&base))) return e;
    hipStream_t s = (hipStream_t)stream;
    const SweepArgs a = make_sweep(height, width, channels, block, overlap_px, robin_alpha,
                                   local_iters);
    const int nb = sweep_partials(a);
    // [transposed mask | norm partials | per-channel sums]; every word the
    // kernels read is written earlier in the same call (the mask-bit launch
    // writes all groups x width words, the sweep one partial per block and
    // channel, the reduction the sums), so nothing is cleared
    unsigned char* p = (unsigned char*)base;
    uint64_t* mb = (uint64_t*)p;
    p += round256((size_t)mask_bit_groups(height) * width * sizeof(uint64_t));
    double* part = (double*)p;
    p += round256((size_t)nb * channels * sizeof(double));
    double* red = (double*)p;
    DDI_HIP(launch_mask_bits(c, height, width, mb, s));
    DDI_HIP(launch_sweep(u_in, mb, u_out, part, nullptr, nullptr, a, s));
    DDI_HIP(launch_reduce(part, nb, channels, channels, red, s));
    if (rsq) {
        DDI_HIP(hipMemcpyAsync(rsq, red, channels * sizeof(double), hipMemcpyDeviceToHost, s));
        DDI_HIP(hipStreamSynchronize(s));
    }
    return DDI_OK;
}

}  // extern "C"
