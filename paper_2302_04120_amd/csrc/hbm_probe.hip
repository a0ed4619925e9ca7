// HBM bandwidth probe used by the benchmark to state the practical ceiling
// of a kernel that reads and writes its state once.  A sweep of simple
// kernels: float4 copies, one-way reads and writes over grids of 256 to 4096
// workgroups with 1 to 8 loads in flight per thread (grid-stride), copies of
// one contiguous chunk per workgroup, nontemporal variants, and copies with
// the two-phase step's access shape (21 planes, one value per plane and
// thread) in plane-major and tile-major order.  Measurement only; not part
// of the LBM library (it allocates its own device buffers).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <vector>

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

// grid-stride copy, U float4 per thread per iteration (all loads, then all
// stores); the loop condition keeps every access below n4
template <int U, bool NT>
__global__ __launch_bounds__(256) void k_copy(const f4v* __restrict__ a, f4v* __restrict__ b,
                                              size_t n4) {
    const size_t T = (size_t)gridDim.x * blockDim.x;
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    for (; i + (U - 1) * T < n4; i += U * T) {
        f4v v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = NT ? __builtin_nontemporal_load(a + i + u * T) : a[i + u * T];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (NT) __builtin_nontemporal_store(v[u], b + i + u * T);
            else b[i + u * T] = v[u];
        }
    }
    for (; i < n4; i += T) b[i] = a[i];
}

// workgroup g copies the contiguous chunk [g C, (g + 1) C) of float4
template <int U, bool NT>
__global__ __launch_bounds__(256) void k_chunk(const f4v* __restrict__ a, f4v* __restrict__ b,
                                               size_t n4, size_t C) {
    const size_t s = blockIdx.x * C, e = s + C < n4 ? s + C : n4;
    size_t i = s + threadIdx.x;
    for (; i + (U - 1) * 256 < e; i += U * 256) {
        f4v v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            v[u] = NT ? __builtin_nontemporal_load(a + i + u * 256) : a[i + u * 256];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (NT) __builtin_nontemporal_store(v[u], b + i + u * 256);
            else b[i + u * 256] = v[u];
        }
    }
    for (; i < e; i += 256) b[i] = a[i];
}

template <int U>
__global__ __launch_bounds__(256) void k_read(const f4v* __restrict__ a, float* __restrict__ sink,
                                              size_t n4) {
    const size_t T = (size_t)gridDim.x * blockDim.x;
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    float s = 0.f;
    for (; i + (U - 1) * T < n4; i += U * T) {
        f4v v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = a[i + u * T];
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u].x + v[u].y + v[u].z + v[u].w;
    }
    for (; i < n4; i += T) s += a[i].x;
    if (s == 1.2345f) sink[0] = s;  // never true for the zero-filled buffer
}

template <int U>
__global__ __launch_bounds__(256) void k_write(f4v* __restrict__ b, size_t n4) {
    const size_t T = (size_t)gridDim.x * blockDim.x;
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    for (; i + (U - 1) * T < n4; i += U * T) {
#pragma unroll
        for (int u = 0; u < U; ++u) b[i + u * T] = f4v{1.f, 2.f, 3.f, 4.f};
    }
    for (; i < n4; i += T) b[i] = f4v{1.f, 2.f, 3.f, 4.f};
}

// 21 planes, node n = global thread (n < N); plane-major: value i of node n
// at i P + n (P >= N); tile-major: the 21 planes of each 256-node tile
// together, value i of node n at (n / 256) 21 256 + i 256 + n % 256 (N a
// multiple of 256)
template <bool TILE_MAJOR, bool NT>
__global__ __launch_bounds__(256) void k_planes(const float* __restrict__ a, float* __restrict__ b,
                                                long long P, long long N) {
    const long long n = blockIdx.x * 256LL + threadIdx.x;
    if (n >= N) return;
    const long long o = TILE_MAJOR ? blockIdx.x * (21LL * 256) + threadIdx.x : n;
    const long long st = TILE_MAJOR ? 256 : P;
    float v[21];
#pragma unroll
    for (int i = 0; i < 21; ++i) v[i] = NT ? __builtin_nontemporal_load(a + o + i * st) : a[o + i * st];
#pragma unroll
    for (int i = 0; i < 21; ++i) {
        if (NT) __builtin_nontemporal_store(v[i], b + o + i * st);
        else b[o + i * st] = v[i];
    }
}

constexpr int kGrids[5] = {256, 512, 1024, 2048, 4096};
constexpr int kProbes = 5 * 7 + 4 + 4;
char g_names[kProbes][48];

}  // namespace

// Number of probes hbm_probe_run measures, and the name of probe i.
extern "C" __attribute__((visibility("default"))) int hbm_probe_count() { return kProbes; }
extern "C" __attribute__((visibility("default"))) const char* hbm_probe_name(int i) {
    return i >= 0 && i < kProbes ? g_names[i] : "";
}

// Runs every probe on two buffers of `bytes` bytes (reps timed repetitions,
// median taken); out[k] (hbm_probe_count() values) receives GB/s of probe k,
// bytes moved (read + written) over the median time.  Needs bytes >= 64 MiB.
// Returns 0, or the HIP error code of the first failing call.
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
    const size_t n4 = bytes / 16;
    const f4v* A4 = (const f4v*)a;
    f4v* B4 = (f4v*)b;
    // 21-plane shapes: N nodes, a multiple of 256, with 21 N floats in a buffer
    const long long N = (long long)(bytes / 4 / 21) / 256 * 256;
    const long long P = N;
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
    int k = 0;
    auto put = [&](double v, const char* fmt, int x, int y) {
        std::snprintf(g_names[k], sizeof g_names[k], fmt, x, y);
        out[k++] = v;
    };
    for (int g : kGrids) {
        put(timeit(cp, [&] { k_copy<1, false><<<g, 256>>>(A4, B4, n4); }), "copy_x%d_grid%d", 1, g);
        put(timeit(cp, [&] { k_copy<4, false><<<g, 256>>>(A4, B4, n4); }), "copy_x%d_grid%d", 4, g);
        put(timeit(cp, [&] { k_copy<4, true><<<g, 256>>>(A4, B4, n4); }), "copy_nt_x%d_grid%d", 4, g);
        put(timeit(one, [&] { k_read<1><<<g, 256>>>(A4, sink, n4); }), "read_x%d_grid%d", 1, g);
        put(timeit(one, [&] { k_read<8><<<g, 256>>>(A4, sink, n4); }), "read_x%d_grid%d", 8, g);
        put(timeit(one, [&] { k_write<1><<<g, 256>>>(B4, n4); }), "write_x%d_grid%d", 1, g);
        put(timeit(one, [&] { k_write<4><<<g, 256>>>(B4, n4); }), "write_x%d_grid%d", 4, g);
    }
    for (int g : {1024, 4096, 16384}) {
        const size_t C = (n4 + g - 1) / g;
        put(timeit(cp, [&] { k_chunk<4, false><<<g, 256>>>(A4, B4, n4, C); }), "copy_chunk_x%d_grid%d",
            4, g);
    }
    {
        const size_t C = (n4 + 2047) / 2048;
        put(timeit(cp, [&] { k_chunk<4, true><<<2048, 256>>>(A4, B4, n4, C); }),
            "copy_chunk_nt_x%d_grid%d", 4, 2048);
    }
    const unsigned gp = (unsigned)(N / 256);
    put(timeit(pl, [&] { k_planes<false, false><<<gp, 256>>>(a, b, P, N); }), "planes%d_plane_major%.0d",
        21, 0);
    put(timeit(pl, [&] { k_planes<false, true><<<gp, 256>>>(a, b, P, N); }),
        "planes%d_plane_major_nt%.0d", 21, 0);
    put(timeit(pl, [&] { k_planes<true, false><<<gp, 256>>>(a, b, P, N); }), "planes%d_tile_major%.0d",
        21, 0);
    put(timeit(pl, [&] { k_planes<true, true><<<gp, 256>>>(a, b, P, N); }),
        "planes%d_tile_major_nt%.0d", 21, 0);
    if (e == hipSuccess) e = hipGetLastError();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (sink) (void)hipFree(sink);
    return (int)e;
}
