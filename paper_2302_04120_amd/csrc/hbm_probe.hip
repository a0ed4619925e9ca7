// HBM bandwidth probe used by the benchmark to state the practical ceiling
// of a kernel that reads and writes its state once: plain and nontemporal
// float4 copies, one-way streams, and a copy with the two-phase step's access
// shape (21 planes, one value per plane per thread).  Measurement only; not
// part of the LBM library (it allocates its own device buffers).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ void k_copy4(const f4v* __restrict__ a, f4v* __restrict__ b, size_t n4) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4;
         i += (size_t)gridDim.x * blockDim.x) {
        f4v v;
        if (NT) v = __builtin_nontemporal_load(a + i); else v = a[i];
        if (NT) __builtin_nontemporal_store(v, b + i); else b[i] = v;
    }
}

__global__ void k_read4(const f4v* __restrict__ a, float* __restrict__ sink, size_t n4) {
    float s = 0.f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4;
         i += (size_t)gridDim.x * blockDim.x) {
        const f4v v = a[i];
        s += v.x + v.y + v.z + v.w;
    }
    if (s == 1.2345f) sink[0] = s;  // never true for the zero-filled buffer
}

__global__ void k_write4(f4v* __restrict__ b, size_t n4) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4;
         i += (size_t)gridDim.x * blockDim.x)
        b[i] = f4v{1.f, 2.f, 3.f, 4.f};
}

// 21 planes of stride P floats, node n = global thread (n < N <= P)
template <bool NT>
__global__ void k_planes(const float* __restrict__ a, float* __restrict__ b, long long P,
                         long long N) {
    const long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (n >= N) return;
    float v[21];
#pragma unroll
    for (int i = 0; i < 21; ++i) v[i] = NT ? __builtin_nontemporal_load(a + i * P + n) : a[i * P + n];
#pragma unroll
    for (int i = 0; i < 21; ++i) {
        if (NT) __builtin_nontemporal_store(v[i], b + i * P + n);
        else b[i * P + n] = v[i];
    }
}

}  // namespace

// Runs every probe on two buffers of `bytes` bytes (reps timed repetitions,
// median taken).  out[k] receives GB/s of probe k in this order:
//   0 copy float4 (grid 1024), 1 copy float4 (grid 8192), 2 copy float4
//   nontemporal (grid 16384), 3 read float4, 4 write float4,
//   5 21-plane step-shaped copy, 6 the same nontemporal.
// Needs bytes >= 64 MiB.  Returns 0, or the HIP error code of the first failing call.
extern "C" __attribute__((visibility("default"))) int hbm_probe_run(size_t bytes, int reps,
                                                                    double* out) {
    if (bytes < (64ull << 20) || reps < 1 || !out) return (int)hipErrorInvalidValue;
    float *a = nullptr, *b = nullptr, *sink = nullptr;
    hipError_t e = hipMalloc(&a, bytes);
    if (e == hipSuccess) e = hipMalloc(&b, bytes);
    if (e == hipSuccess) e = hipMalloc(&sink, 256);
    if (e == hipSuccess) e = hipMemset(a, 0, bytes);
    if (e == hipSuccess) e = hipMemset(b, 0, bytes);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const size_t n = bytes / 4, n4 = n / 4;
    long long P = (long long)(n / 21) - 64;
    P -= P % 64;
    const long long N = P - 16448;
    auto timeit = [&](double moved, auto launch) -> double {
        if (e != hipSuccess) return 0.0;
        launch();
        e = hipDeviceSynchronize();
        std::vector<float> t;
        for (int r = 0; r < reps && e == hipSuccess; ++r) {
            e = hipEventRecord(e0);
            launch();
            if (e == hipSuccess) e = hipEventRecord(e1);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            t.push_back(ms);
        }
        if (e != hipSuccess || t.empty()) return 0.0;
        std::sort(t.begin(), t.end());
        return moved / (t[t.size() / 2] * 1e-3) / 1e9;
    };
    const double cp = 2.0 * (double)bytes, one = (double)bytes, pl = 2.0 * 21 * 4 * (double)N;
    out[0] = timeit(cp, [&] { k_copy4<false><<<1024, 256>>>((const f4v*)a, (f4v*)b, n4); });
    out[1] = timeit(cp, [&] { k_copy4<false><<<8192, 256>>>((const f4v*)a, (f4v*)b, n4); });
    out[2] = timeit(cp, [&] { k_copy4<true><<<16384, 256>>>((const f4v*)a, (f4v*)b, n4); });
    out[3] = timeit(one, [&] { k_read4<<<8192, 256>>>((const f4v*)a, sink, n4); });
    out[4] = timeit(one, [&] { k_write4<<<8192, 256>>>((f4v*)b, n4); });
    const unsigned gp = (unsigned)((N + 255) / 256);
    out[5] = timeit(pl, [&] { k_planes<false><<<gp, 256>>>(a, b, P, N); });
    out[6] = timeit(pl, [&] { k_planes<true><<<gp, 256>>>(a, b, P, N); });
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (sink) (void)hipFree(sink);
    return (int)e;
}
