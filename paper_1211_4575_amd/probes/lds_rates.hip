// Throughput of the LDS instructions that bound the particle kernel, on one gfx950 GPU:
// 64-bit integer atomic adds in the current deposit's address pattern (each lane owns one
// cell of a 4x4x4 tile and adds to a 4x5x5 window of a current block with row stride 12 and
// plane stride 128, as the kernel's layout), the same with a fraction of lanes whose window
// is shifted by one node, 32- and 64-bit atomic adds to consecutive addresses, and paired
// 32-bit reads (the gather's instruction).  Prints clocks per wavefront instruction per CU
// (256 CUs at 2.4 GHz).  Every LDS index is checked on the host against the array size
// before any launch.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

namespace {

constexpr int QN = 6144;  // 64-bit LDS words per workgroup (48 KiB)
constexpr int CROW = 12, CPLANE = 128;
constexpr int BLOCKS = 256 * 20, ITERS = 32;

#define CHECK(x)                                                                    \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
            return 1;                                                               \
        }                                                                           \
    } while (0)

// 100 adds per lane per iteration: the deposit's J_x block of one particle
__global__ void __launch_bounds__(256) k_deposit_u64(const int* __restrict__ base_tab, float* out, int iters) {
    __shared__ unsigned long long q[QN];
    for (int i = threadIdx.x; i < QN; i += 256) q[i] = 0;
    __syncthreads();
    const int base = base_tab[threadIdx.x];
    for (int it = 0; it < iters; ++it) {
        const unsigned long long v = (unsigned long long)(it + 1);
#pragma unroll
        for (int e = 0; e < 5; ++e)
#pragma unroll
            for (int b = 0; b < 5; ++b)
#pragma unroll
                for (int a = 0; a < 4; ++a) atomicAdd(&q[base + a + b * CROW + e * CPLANE], v);
    }
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (float)q[5];
}

// 100 adds per lane per iteration to consecutive addresses (lane l: word l, then + 64 k)
template <typename T>
__global__ void __launch_bounds__(256) k_contiguous(float* out, int iters) {
    __shared__ T q[QN];
    for (int i = threadIdx.x; i < QN; i += 256) q[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 100; ++k) atomicAdd(&q[lane + 64 * (k % 64)], (T)(it + 1));
    }
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (float)q[5];
}

// 100 paired 32-bit reads per lane per iteration (two floats 8 apart, lane-consecutive)
__global__ void __launch_bounds__(256) k_read2(float* out, int iters) {
    __shared__ float f[2 * QN];
    for (int i = threadIdx.x; i < 2 * QN; i += 256) f[i] = (float)i;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    float acc = 0.f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 100; ++k) {
            const int i = lane + 72 * ((k + it) % 64);  // < 72 * 64 + 64 + 8 <= 2 * QN
            acc += f[i] * f[i + 8];
        }
    }
    out[blockIdx.x * 256 + threadIdx.x] = acc;
}

double clk_per_instr(float ms, double lane_ops) {
    const double per_clk_cu = lane_ops / (ms * 1e-3) / 256.0 / 2.4e9;
    return 64.0 / per_clk_cu;
}

}  // namespace

int main() {
    float* out = nullptr;
    int* dtab = nullptr;
    CHECK(hipMalloc(&out, (size_t)BLOCKS * 256 * sizeof(float)));
    CHECK(hipMalloc(&dtab, 256 * sizeof(int)));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const double lane_ops = (double)BLOCKS * 256 * ITERS * 100;
    auto timed = [&](auto launch) -> float {
        float ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {  // the first launch warms up
            (void)hipEventRecord(e0);
            launch();
            (void)hipEventRecord(e1);
            (void)hipEventSynchronize(e1);
            (void)hipEventElapsedTime(&ms, e0, e1);
        }
        return ms;
    };

    std::printf("%-44s %9s %12s\n", "pattern", "ms", "clk/instr");
    std::mt19937 rng(7);
    for (double shift : {0.0, 0.07, 0.25}) {
        // lane l of each wavefront owns local cell (l % 4, l / 4 % 4, l / 16) of a 4x4x4
        // tile; its window starts two nodes below the cell, or one node higher along an axis
        // with probability `shift`
        std::vector<int> tab(256);
        std::uniform_real_distribution<double> U(0, 1);
        int mx = 0;
        for (int t = 0; t < 256; ++t) {
            const int l = t & 63;
            const int c[3] = {l % 4, l / 4 % 4, l / 16};
            int b = 0;
            const int stride[3] = {1, CROW, CPLANE};
            for (int d = 0; d < 3; ++d) b += (c[d] + (U(rng) < shift ? 1 : 0)) * stride[d];
            tab[t] = b;
            const int last = b + 3 + 4 * CROW + 4 * CPLANE;
            mx = last > mx ? last : mx;
        }
        if (mx >= QN) {
            std::printf("window pattern exceeds the LDS block (%d >= %d): skipped\n", mx, QN);
            continue;
        }
        CHECK(hipMemcpy(dtab, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice));
        const float ms = timed([&] {
            hipLaunchKernelGGL(k_deposit_u64, dim3(BLOCKS), dim3(256), 0, 0, dtab, out, ITERS);
        });
        char name[64];
        std::snprintf(name, sizeof name, "ds_add_u64 deposit window, %2.0f%% lanes shifted", 100.0 * shift);
        std::printf("%-44s %9.3f %12.1f\n", name, ms, clk_per_instr(ms, lane_ops));
    }
    {
        const float ms = timed([&] {
            hipLaunchKernelGGL(k_contiguous<unsigned long long>, dim3(BLOCKS), dim3(256), 0, 0, out, ITERS);
        });
        std::printf("%-44s %9.3f %12.1f\n", "ds_add_u64 consecutive words", ms, clk_per_instr(ms, lane_ops));
    }
    {
        const float ms = timed([&] {
            hipLaunchKernelGGL(k_contiguous<unsigned int>, dim3(BLOCKS), dim3(256), 0, 0, out, ITERS);
        });
        std::printf("%-44s %9.3f %12.1f\n", "ds_add_u32 consecutive words", ms, clk_per_instr(ms, lane_ops));
    }
    {
        const float ms = timed([&] { hipLaunchKernelGGL(k_read2, dim3(BLOCKS), dim3(256), 0, 0, out, ITERS); });
        std::printf("%-44s %9.3f %12.1f\n", "ds_read2_b32 (two floats per lane)", ms, clk_per_instr(ms, lane_ops));
    }
    CHECK(hipDeviceSynchronize());
    CHECK(hipGetLastError());
    std::printf("status ok\n");
    (void)hipFree(out);
    (void)hipFree(dtab);
    return 0;
}
