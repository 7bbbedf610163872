// atomic_rates.hip -- throughput of the atomic additions the step's design
// chooses between, on the device it runs on: global FP32 and FP64 adds
// (each lane to its own scattered cache line, or lanes of a wave to
// consecutive addresses) and LDS FP32 and FP64 adds (lanes to distinct
// addresses).  One workgroup, then 256 and 2048 workgroups of 384 threads,
// 256 additions per thread.  A measurement program, not part of the library.
#include <hip/hip_runtime.h>

#include <cstdio>

#define CHECK(x)                                                                        \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                         \
            std::printf("%s: %s\n", #x, hipGetErrorString(e_));                         \
            return 1;                                                                   \
        }                                                                               \
    } while (0)

constexpr int kThreads = 384;
constexpr int kIters = 256;
constexpr int kLds = kThreads * 4;

// integer hash (spreads lane addresses over the array)
__device__ __forceinline__ unsigned mix(unsigned x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// f has mask + 1 elements (a power of two): every index is in bounds
template <typename T, bool SCATTER>
__global__ __launch_bounds__(kThreads) void k_global(T *f, unsigned mask) {
    const unsigned g = blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = 0; i < kIters; ++i) {
        const unsigned idx = SCATTER ? (mix(g * 977u + i * 131071u) & mask)
                                     : (((blockIdx.x * kIters + i) * blockDim.x + threadIdx.x) & mask);
        unsafeAtomicAdd(f + idx, (T)1);
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_lds(T *out) {
    __shared__ T s[kLds];
    for (int i = threadIdx.x; i < kLds; i += blockDim.x) s[i] = 0;
    __syncthreads();
    for (int i = 0; i < kIters; ++i) {
        const int idx = (threadIdx.x * 3 + i * 7) % kLds;
        __hip_atomic_fetch_add(s + idx, (T)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

template <typename L>
static float time_ms(L launch) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    launch();
    (void)hipDeviceSynchronize();
    (void)hipEventRecord(a);
    for (int r = 0; r < 5; ++r) launch();
    (void)hipEventRecord(b);
    (void)hipEventSynchronize(b);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / 5;
}

int main() {
    const size_t n = size_t(1) << 26;
    float *f32 = nullptr;
    double *f64 = nullptr;
    CHECK(hipMalloc(&f32, n * sizeof(float)));
    CHECK(hipMalloc(&f64, n * sizeof(double)));
    CHECK(hipMemset(f32, 0, n * sizeof(float)));
    CHECK(hipMemset(f64, 0, n * sizeof(double)));
    const unsigned mask = (unsigned)(n - 1);
    std::printf("%-24s %8s %10s %14s\n", "addition", "blocks", "ms", "G additions/s");
    for (int blocks : {1, 256, 2048}) {
        const double adds = (double)blocks * kThreads * kIters;
        const auto row = [&](const char *name, float ms) {
            std::printf("%-24s %8d %10.3f %14.2f\n", name, blocks, ms, adds / ms / 1e6);
        };
        row("global f32 scattered", time_ms([&] {
                hipLaunchKernelGGL((k_global<float, true>), dim3(blocks), dim3(kThreads), 0, 0, f32, mask);
            }));
        row("global f32 consecutive", time_ms([&] {
                hipLaunchKernelGGL((k_global<float, false>), dim3(blocks), dim3(kThreads), 0, 0, f32, mask);
            }));
        row("global f64 scattered", time_ms([&] {
                hipLaunchKernelGGL((k_global<double, true>), dim3(blocks), dim3(kThreads), 0, 0, f64, mask);
            }));
        row("global f64 consecutive", time_ms([&] {
                hipLaunchKernelGGL((k_global<double, false>), dim3(blocks), dim3(kThreads), 0, 0, f64, mask);
            }));
        row("LDS f32", time_ms([&] {
                hipLaunchKernelGGL((k_lds<float>), dim3(blocks), dim3(kThreads), 0, 0, f32);
            }));
        row("LDS f64", time_ms([&] {
                hipLaunchKernelGGL((k_lds<double>), dim3(blocks), dim3(kThreads), 0, 0, f64);
            }));
    }
    CHECK(hipGetLastError());
    CHECK(hipFree(f32));
    CHECK(hipFree(f64));
    return 0;
}
