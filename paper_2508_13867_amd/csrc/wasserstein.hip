// 1-Wasserstein distance between the numerical statistical solutions of two
// jobs (Sec. "Taylor--Green vortex flow with four-dimensional uncertain
// initial velocity perturbation", Eq. of W_1): each job's law of a field QoI
// is the weighted empirical measure of all its values (value o of sample j
// carries weight a_j / n_out); for two measures on the real line
//   W_1 = integral_0^1 |Q_a(p) - Q_b(p)| dp
// with Q the quantile functions. Both laws are sorted on the device (hipCUB
// radix sort of value/weight pairs), their cumulative weights formed (hipCUB
// inclusive scan), and every value of a accumulates |x - y| times the overlap
// of its probability interval with those of the values y of b (found by
// binary search), in compensated FP64.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "uq_job.h"

namespace uqi {

namespace {

struct NSumW {
    double s = 0.0, c = 0.0;
    __device__ inline void add(double x) {
        const double t = s + x;
        c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    }
};

// gather the field values of every sample, scaled, with weight a_j / n_out
__global__ void k_w1_gather(const double *M, int64_t S, int64_t n_out, int64_t ld, const double *a, double scale,
                            double *keys, double *wts) {
    const int64_t L = S * n_out;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < L; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / n_out, o = e - j * n_out;
        keys[e] = M[j * ld + o] * scale;
        wts[e] = a[j] / (double)n_out;
    }
}

// first index j in [0, n) with P[j] > p (P nondecreasing), or n
__device__ inline int64_t upper(const double *P, int64_t n, double p) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (P[mid] > p) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// partial sums of |x_i - y_j| * overlap over intervals i of a, per block
__global__ __launch_bounds__(256) void k_w1_overlap(const double *xa, const double *Pa, int64_t na, const double *xb,
                                                    const double *Pb, int64_t nb, double *partial) {
    NSumW acc;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na; i += (int64_t)gridDim.x * blockDim.x) {
        const double lo = i == 0 ? 0.0 : Pa[i - 1];
        const double hi = i == na - 1 ? 1.0 : Pa[i];
        if (!(hi > lo)) continue;
        // the last interval of b ends at 1 whatever its rounded cumulative
        // weight, so the search runs over the first nb - 1 ends only
        for (int64_t j = upper(Pb, nb - 1, lo); j < nb; ++j) {
            const double blo = j == 0 ? 0.0 : Pb[j - 1];
            const double bhi = j == nb - 1 ? 1.0 : Pb[j];
            if (blo >= hi) break;
            const double ov = fmin(hi, bhi) - fmax(lo, blo);
            if (ov > 0.0) acc.add(fabs(xa[i] - xb[j]) * ov);
        }
    }
    __shared__ double sh[2][256];
    sh[0][threadIdx.x] = acc.s;
    sh[1][threadIdx.x] = acc.c;
    __syncthreads();
    if (threadIdx.x == 0) {
        NSumW b;
        for (int t = 0; t < (int)blockDim.x; ++t) {
            b.add(sh[0][t]);
            b.add(sh[1][t]);
        }
        partial[2 * blockIdx.x] = b.s;
        partial[2 * blockIdx.x + 1] = b.c;
    }
}

__global__ void k_w1_finish(const double *partial, int nblocks, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    NSumW b;
    for (int t = 0; t < 2 * nblocks; ++t) b.add(partial[t]);
    out[0] = b.s + b.c;
}

}  // namespace

// Device buffers of one W_1 evaluation, taken from job `owner`. Whatever is
// still held when the guard goes out of scope (every early return) is given
// back after the owner's stream has drained, so no error path leaks a block
// or frees one that a queued kernel still reads.
struct W1Buffers {
    Job *owner;
    std::vector<void *> held;
    explicit W1Buffers(Job *o) : owner(o) {}
    W1Buffers(const W1Buffers &) = delete;
    W1Buffers &operator=(const W1Buffers &) = delete;
    void *take(size_t bytes) {
        void *p = owner->dalloc(bytes);
        if (p) held.push_back(p);
        return p;
    }
    void give_back(void *p) {  // caller has ordered the stream already
        for (size_t i = 0; i < held.size(); ++i)
            if (held[i] == p) {
                owner->dfree(p);
                held.erase(held.begin() + (long)i);
                return;
            }
    }
    ~W1Buffers() {
        if (held.empty()) return;
        (void)hipStreamSynchronize(owner->stream);
        (void)hipGetLastError();
        for (void *p : held) owner->dfree(p);
    }
};

// sorted values and cumulative weights of one job's law, in buffers of `buf`
static uq_status build_law(W1Buffers &buf, Job *src, int qoi, double scale, double **x_sorted, double **P,
                           int64_t *n) {
    Job *owner = buf.owner;
    const double *M;
    int64_t n_out, ld;
    uq_status st = src->sample_values(qoi, &M, &n_out, &ld);
    if (st != UQ_OK) return st;
    const int64_t L = src->S * n_out;
    if (L >= ((int64_t)1 << 31)) return fail(UQ_EINVAL, "law too large for one sort");
    double *a_dev = (double *)buf.take(sizeof(double) * src->S);
    double *k0 = (double *)buf.take(sizeof(double) * L), *w0 = (double *)buf.take(sizeof(double) * L);
    double *k1 = (double *)buf.take(sizeof(double) * L), *w1 = (double *)buf.take(sizeof(double) * L);
    if (!a_dev || !k0 || !w0 || !k1 || !w1) return fail(UQ_ENOMEM, "out of device memory for the W1 sort");
    hipStream_t s = owner->stream;
    // values are produced on src's stream; order owner's stream after it
    UQ_HIP_TRY(hipEventRecord(src->ev_out, src->stream));
    UQ_HIP_TRY(hipStreamWaitEvent(s, src->ev_out, 0));
    UQ_HIP_TRY(hipMemcpyAsync(a_dev, src->rule.a.data(), sizeof(double) * src->S, hipMemcpyHostToDevice, s));
    k_w1_gather<<<(unsigned)std::min<int64_t>((L + 255) / 256, 65536), 256, 0, s>>>(M, src->S, n_out, ld, a_dev,
                                                                                      scale, k0, w0);
    UQ_HIP_TRY(hipGetLastError());
    size_t tb = 0, tb2 = 0;
    UQ_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, k0, k1, w0, w1, (int)L, 0, 64, s));
    UQ_HIP_TRY(hipcub::DeviceScan::InclusiveSum(nullptr, tb2, w1, w0, (int)L, s));
    void *tmp = buf.take(std::max(tb, tb2));
    if (!tmp) return fail(UQ_ENOMEM, "out of device memory for the W1 sort");
    UQ_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(tmp, tb, k0, k1, w0, w1, (int)L, 0, 64, s));
    UQ_HIP_TRY(hipcub::DeviceScan::InclusiveSum(tmp, tb2, w1, w0, (int)L, s));
    UQ_HIP_TRY(hipStreamSynchronize(s));  // host copy of a_j must stay alive until here
    for (void *p : {tmp, (void *)a_dev, (void *)k0, (void *)w1}) buf.give_back(p);
    *x_sorted = k1;  // sorted values
    *P = w0;         // cumulative weights
    *n = L;
    return UQ_OK;
}

}  // namespace uqi

using namespace uqi;

extern "C" uq_status uq_wasserstein1(uq_job *a, uq_job *b, int32_t qoi, double scale_a, double scale_b, double *w1) {
    if (!a || !b || !w1) return fail(UQ_EINVAL, "null argument");
    if (qoi != UQ_QOI_VEL && qoi != UQ_QOI_RHO && qoi != UQ_QOI_SPEED)
        return fail(UQ_EINVAL, "W1 compares field QoIs (VEL, RHO, SPEED)");
    if (a->dev.device != b->dev.device) return fail(UQ_EINVAL, "jobs on different devices");
    for (Job *j : {(Job *)a, (Job *)b})
        for (double w : j->rule.a)
            if (w < 0.0) return fail(UQ_EINVAL, "W1 needs a rule with nonnegative weights");
    UQ_HIP_TRY(hipSetDevice(a->dev.device));
    uq_status st = a->enter();
    if (st != UQ_OK) return st;
    if (b != a) {
        st = b->enter();
        if (st != UQ_OK) return st;
    }
    double *xa = nullptr, *Pa = nullptr, *xb = nullptr, *Pb = nullptr;
    int64_t na = 0, nb = 0;
    {
        W1Buffers buf(a);  // every buffer below goes back to job a on return
        st = build_law(buf, a, qoi, scale_a, &xa, &Pa, &na);
        if (st == UQ_OK) st = build_law(buf, b, qoi, scale_b, &xb, &Pb, &nb);
        if (st != UQ_OK) return st;
        // W_1 is symmetric: the larger law takes the outer loop, so each
        // thread meets about one interval of the other
        if (nb > na) {
            std::swap(xa, xb);
            std::swap(Pa, Pb);
            std::swap(na, nb);
        }
        const int nblocks = (int)std::min<int64_t>((na + 255) / 256, 4096);
        double *partial = (double *)buf.take(sizeof(double) * (2 * nblocks + 1));
        if (!partial) return fail(UQ_ENOMEM, "out of device memory");
        k_w1_overlap<<<nblocks, 256, 0, a->stream>>>(xa, Pa, na, xb, Pb, nb, partial);
        UQ_HIP_TRY(hipGetLastError());
        k_w1_finish<<<1, 64, 0, a->stream>>>(partial, nblocks, partial + 2 * nblocks);
        UQ_HIP_TRY(hipGetLastError());
        UQ_HIP_TRY(hipMemcpyAsync(w1, partial + 2 * nblocks, sizeof(double), hipMemcpyDeviceToHost, a->stream));
        UQ_HIP_TRY(hipStreamSynchronize(a->stream));
        for (void *p : {(void *)xa, (void *)Pa, (void *)xb, (void *)Pb, (void *)partial}) buf.give_back(p);
    }
    st = a->leave();
    if (st == UQ_OK && b != a) {
        // b's stream must not run ahead of the reads of its fields
        UQ_HIP_TRY(hipEventRecord(a->ev_out, a->stream));
        UQ_HIP_TRY(hipStreamWaitEvent(b->stream, a->ev_out, 0));
    }
    return st;
}
