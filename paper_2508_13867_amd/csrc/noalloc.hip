// Allocation-free statistics: uq_moments_noalloc, a variant of uq_moments for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc). It runs the same
// kernels as uq_moments; their intermediates -- the per-sample scalar QoIs,
// the moment outputs and the non-finite flag -- live in one file-scope
// device array per GPU instead of buffers the job allocates on its first
// statistics call.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "uq_job.h"

namespace uqi {

namespace {

constexpr size_t kScratchBytes = (size_t)UQ_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// Each GPU the library runs on holds its own copy of this array until the
// process ends. Host code names it only in hipGetSymbolAddress: on the host
// the name is a stand-in, not a device address.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
    std::mutex use;       // calls on one device share the array: one at a time
    void *ptr = nullptr;  // device address of `scratch` on this device
};
DeviceScratch g_dev[kMaxDevices];

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// Carve the statistics buffers of one call out of `base` (null: sizes only);
// returns the bytes used. Layout: qoi[S][4], M[S], flag, out[(K+3) n_out]
// (the moments of a field are formed from the populations: no per-sample
// field buffer).
size_t carve(const Job &j, int qoi, unsigned char *base, StatBufs *b) {
    const int64_t S = j.S, n_out = qoi_width(j.p, qoi);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *p = base ? base + off : nullptr;
        off += up256(bytes);
        return p;
    };
    unsigned char *q = take(sizeof(double) * 4 * S);
    unsigned char *M = take(sizeof(double) * S);
    unsigned char *flag = take(sizeof(int64_t));
    unsigned char *out = take(sizeof(double) * (size_t)((j.K > 0 ? j.K : 0) + 3) * n_out);
    if (b) {
        b->qoi = (double *)q;
        b->M = (double *)M;
        b->flag = (int64_t *)flag;
        b->out = (double *)out;
        b->fields = nullptr;
    }
    return off;
}

}  // namespace

}  // namespace uqi

using namespace uqi;

extern "C" uq_status uq_moments_noalloc(uq_job *j, int32_t qoi, uq_moments_out *out) {
    if (!j || !out) return fail(UQ_EINVAL, "null argument");
    if (qoi_width(j->p, qoi) == 0) return fail(UQ_EINVAL, "unknown QoI");
    const int dev = j->dev.device;
    if (dev < 0 || dev >= kMaxDevices) return fail(UQ_EINVAL, "device ordinal out of range for uq_moments_noalloc");
    const size_t need = carve(*j, qoi, nullptr, nullptr);
    if (need > kScratchBytes)
        return fail(UQ_EINVAL, "uq_moments_noalloc: this QoI of this job needs " + std::to_string(need) +
                                   " B of scratch, more than the library's fixed " + std::to_string(kScratchBytes) +
                                   " B (use uq_moments)");
    UQ_HIP_TRY(hipSetDevice(dev));
    DeviceScratch &ds = g_dev[dev];
    // held until the results are on the host: the next call may then reuse
    // the array (every kernel of the path overwrites what it later reads, so
    // nothing needs clearing between calls)
    std::lock_guard<std::mutex> lk(ds.use);
    if (!ds.ptr) {
        void *p = nullptr;
        UQ_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(UQ_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        ds.ptr = p;
    }
    StatBufs b;
    carve(*j, qoi, (unsigned char *)ds.ptr, &b);
    return j->moments_in(b, qoi, out);
}
