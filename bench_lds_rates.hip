// Instruction-rate probe for the particle kernel's cost model on one gfx950 GPU (measurement
// only; not part of libpp).  Built and run by `python bench.py --lds-probe`.
//
// Prints clocks per wavefront instruction per CU (256 CUs at 2.4 GHz) for:
//   * 64-bit integer LDS atomic adds in the current deposit's address pattern (lane l owns
//     cell (l%4, l/4%4, l/16) of a 4x4x4 tile and adds to a 4x5x5 window of a block with row
//     stride 12 and plane stride 128), also with a fraction of windows shifted by one node and
//     with only 4 of every 16 lanes active;
//   * the same pattern as 32-bit float atomic adds and as plain 64-bit stores;
//   * atomic adds and reads to consecutive words (the LDS unit's own rates);
//   * the gather's paired 32-bit reads in its real pattern (4x4 rows of 4 floats per lane,
//     row stride 10, plane stride 90 floats) and 128-bit aligned reads;
//   * FP32 and FP64 fused multiply-adds and FP32 adds whose operand comes from another lane of
//     the same row of 16 (DPP row shift), i.e. the vector ALU rates.
// Every LDS index is checked on the host against the array size before any launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

namespace {

constexpr int QN = 6144;  // 64-bit LDS words per workgroup (48 KiB)
constexpr int CROW = 12, CPLANE = 128;
constexpr int FROW = 10, FPLANE = 90;  // gather field tile strides (floats)
constexpr int BLOCKS = 256 * 20, ITERS = 32;

#define CHECK(x)                                                                    \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess) {                                                     \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
            return 1;                                                               \
        }                                                                           \
    } while (0)

// 100 adds per lane per iteration: the deposit's J_x block of one particle.  Lanes whose
// bit in `active` is clear skip the adds (exec-masked instructions).
template <typename T>
__global__ void __launch_bounds__(256) k_deposit(const int* __restrict__ base_tab, float* out, int iters,
                                                 unsigned long long active) {
    __shared__ T q[QN * sizeof(unsigned long long) / sizeof(T)];
    for (int i = threadIdx.x; i < QN * (int)(sizeof(unsigned long long) / sizeof(T)); i += 256) q[i] = 0;
    __syncthreads();
    const int base = base_tab[threadIdx.x];
    const bool on = (active >> (threadIdx.x & 63)) & 1ull;
    if (on) {
        for (int it = 0; it < iters; ++it) {
            const T v = (T)(it + 1);
#pragma unroll
            for (int e = 0; e < 5; ++e)
#pragma unroll
                for (int b = 0; b < 5; ++b)
#pragma unroll
                    for (int a = 0; a < 4; ++a) atomicAdd(&q[base + a + b * CROW + e * CPLANE], v);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (float)q[5];
}

// 100 plain 64-bit stores per lane per iteration in the deposit pattern (distinct addresses
// for every lane of an instruction when no window is shifted)
__global__ void __launch_bounds__(256) k_deposit_store(const int* __restrict__ base_tab, float* out, int iters) {
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
                for (int a = 0; a < 4; ++a) q[(it & 1) * 2048 + base + a + b * CROW + e * CPLANE] = v + a;
        asm volatile("" ::: "memory");  // keep every iteration's stores
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

// 100 128-bit aligned reads per lane per iteration (lane-consecutive float4)
__global__ void __launch_bounds__(256) k_read128(float* out, int iters) {
    __shared__ float4 f[QN / 2];
    for (int i = threadIdx.x; i < QN / 2; i += 256) f[i] = make_float4(i, i + 1, i + 2, i + 3);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    float acc = 0.f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 100; ++k) {
            const float4 v = f[lane + 64 * ((k + it) % 48)];  // < 64 * 48 = QN / 2
            acc += v.x * v.y + v.z * v.w;
        }
    }
    out[blockIdx.x * 256 + threadIdx.x] = acc;
}

// The gather of one component of one particle (cubic weights): 16 rows of 4 floats around the
// lane's cell, row stride FROW, plane stride FPLANE; 6 components per iteration (96 rows).
__global__ void __launch_bounds__(256) k_gather(const int* __restrict__ fbase_tab, float* out, int iters) {
    __shared__ float f[2 * QN];
    for (int i = threadIdx.x; i < 2 * QN; i += 256) f[i] = (float)(i & 255);
    __syncthreads();
    const int base = fbase_tab[threadIdx.x];
    float acc = 0.f;
    for (int it = 0; it < iters; ++it) {
        const float w = (float)(it & 3) * 0.25f;
#pragma unroll
        for (int comp = 0; comp < 6; ++comp) {
            const float* F = f + base + comp * 1000;
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const float* row = F + c * FPLANE + b * FROW;
                    acc += row[0] * w + row[1] * (1.f - w) + row[2] * w + row[3];
                }
        }
    }
    out[blockIdx.x * 256 + threadIdx.x] = acc;
}

// 128 FP32 (or FP64) fused multiply-adds per lane per iteration over 8 independent chains
template <typename T>
__global__ void __launch_bounds__(256) k_fma(float* out, int iters, T x) {
    T a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (T)(threadIdx.x + j);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k)
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = a[j] * x + (T)0.5;
    }
    T s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += a[j];
    out[blockIdx.x * 256 + threadIdx.x] = (float)s;
}

// 128 FP32 adds per lane per iteration whose first operand comes from the lane one place lower
// in its row of 16 (DPP row_shr:1, zero for the row's first lane)
__global__ void __launch_bounds__(256) k_dpp_add(float* out, int iters, float x) {
    const float w = x * (float)(threadIdx.x & 1);  // a per-lane operand (a VGPR)
    float a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (float)(threadIdx.x + j) * 1e-3f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int s = __builtin_amdgcn_update_dpp(0, __float_as_int(a[j]), 0x111, 0xf, 0xf, true);
                a[j] = __int_as_float(s) * w + a[j];
            }
    }
    float s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += a[j];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}


// Realistic wavefront patterns of the particle kernel: each wavefront takes one 64-particle
// chunk of a tile's particle order (table of 64 LDS bases per chunk) and issues the deposit's
// 100 atomic adds (window of 4x5x5 nodes) or the gather's 192 paired reads per lane.
__global__ void __launch_bounds__(256) k_chunk_deposit(const int* __restrict__ tab, int nchunks, float* out,
                                                       int iters, int crow, int cplane) {
    __shared__ unsigned long long q[QN];
    for (int i = threadIdx.x; i < QN; i += 256) q[i] = 0;
    __syncthreads();
    const int chunk = (int)((blockIdx.x * 4 + (threadIdx.x >> 6)) % (unsigned)nchunks);
    const int base = tab[chunk * 64 + (threadIdx.x & 63)];
    for (int it = 0; it < iters; ++it) {
        const unsigned long long v = (unsigned long long)(it + 1);
#pragma unroll
        for (int e = 0; e < 5; ++e)
#pragma unroll
            for (int b = 0; b < 5; ++b)
#pragma unroll
                for (int a = 0; a < 4; ++a) atomicAdd(&q[base + a + b * crow + e * cplane], v);
    }
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (float)q[5];
}

__global__ void __launch_bounds__(256) k_chunk_gather(const int* __restrict__ tab, int nchunks, float* out, int iters,
                                                      int frow, int fplane) {
    __shared__ float f[2 * QN];
    for (int i = threadIdx.x; i < 2 * QN; i += 256) f[i] = (float)(i & 255);
    __syncthreads();
    const int chunk = (int)((blockIdx.x * 4 + (threadIdx.x >> 6)) % (unsigned)nchunks);
    const int base = tab[chunk * 64 + (threadIdx.x & 63)];
    float acc = 0.f;
    for (int it = 0; it < iters; ++it) {
        const float w = (float)(it & 3) * 0.25f;
#pragma unroll
        for (int comp = 0; comp < 6; ++comp) {
            const float* F = f + base + comp * 1600;
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const float* row = F + c * fplane + b * frow;
                    acc += row[0] * w + row[1] * (1.f - w) + row[2] * w + row[3];
                }
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
    auto row = [&](const char* name, float ms, double ops) {
        std::printf("%-84s %9.3f %10.1f\n", name, ms, clk_per_instr(ms, ops));
        std::fflush(stdout);
    };

    std::printf("%-84s %9s %10s\n", "pattern", "ms", "clk/instr");
    std::mt19937 rng(7);
    // deposit window tables: lane l of each wavefront owns local cell (l % 4, l / 4 % 4, l / 16)
    // of a 4x4x4 tile; its window starts at the cell, or one node higher along an axis with
    // probability `shift`
    auto window_table = [&](double shift, std::vector<int>& tab) -> bool {
        tab.assign(256, 0);
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
        return mx < QN;  // the float form uses 2 * QN words: also in range
    };
    std::vector<int> tab;
    for (double shift : {0.0, 0.07, 0.25}) {
        if (!window_table(shift, tab)) {
            std::printf("window pattern exceeds the LDS block: skipped\n");
            continue;
        }
        CHECK(hipMemcpy(dtab, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice));
        char name[80];
        float ms = timed([&] {
            hipLaunchKernelGGL(k_deposit<unsigned long long>, dim3(BLOCKS), dim3(256), 0, 0, dtab, out, ITERS,
                               ~0ull);
        });
        std::snprintf(name, sizeof name, "ds_add_u64 deposit window, %2.0f%% lanes shifted", 100.0 * shift);
        row(name, ms, lane_ops);
        ms = timed([&] {
            hipLaunchKernelGGL(k_deposit<float>, dim3(BLOCKS), dim3(256), 0, 0, dtab, out, ITERS, ~0ull);
        });
        std::snprintf(name, sizeof name, "ds_add_f32 deposit window, %2.0f%% lanes shifted", 100.0 * shift);
        row(name, ms, lane_ops);
        if (shift == 0.0) {
            // 4 of every 16 lanes active: the cost of an exec-masked instruction, per
            // wavefront instruction issued (lane_ops counts 64 lanes per instruction)
            ms = timed([&] {
                hipLaunchKernelGGL(k_deposit<unsigned long long>, dim3(BLOCKS), dim3(256), 0, 0, dtab, out, ITERS,
                                   0xF000F000F000F000ull);
            });
            row("ds_add_u64 deposit window, 16 of 64 lanes active", ms, lane_ops);
            ms = timed([&] {
                hipLaunchKernelGGL(k_deposit_store, dim3(BLOCKS), dim3(256), 0, 0, dtab, out, ITERS);
            });
            row("ds_write_b64 deposit window (plain stores)", ms, lane_ops);
        }
    }
    {
        float ms = timed([&] {
            hipLaunchKernelGGL(k_contiguous<unsigned long long>, dim3(BLOCKS), dim3(256), 0, 0, out, ITERS);
        });
        row("ds_add_u64 consecutive words", ms, lane_ops);
        ms = timed([&] {
            hipLaunchKernelGGL(k_contiguous<unsigned int>, dim3(BLOCKS), dim3(256), 0, 0, out, ITERS);
        });
        row("ds_add_u32 consecutive words", ms, lane_ops);
        ms = timed([&] { hipLaunchKernelGGL(k_contiguous<float>, dim3(BLOCKS), dim3(256), 0, 0, out, ITERS); });
        row("ds_add_f32 consecutive words", ms, lane_ops);
        ms = timed([&] { hipLaunchKernelGGL(k_read2, dim3(BLOCKS), dim3(256), 0, 0, out, ITERS); });
        row("ds_read2_b32 (two floats per lane)", ms, lane_ops);
        ms = timed([&] { hipLaunchKernelGGL(k_read128, dim3(BLOCKS), dim3(256), 0, 0, out, ITERS); });
        row("ds_read_b128 (aligned float4 per lane)", ms, lane_ops);
    }
    {
        // gather: lane l's cell (l%4, l/4%4, l/16); its 4x4x4 support starts one node below
        std::vector<int> ft(256);
        int mx = 0;
        for (int t = 0; t < 256; ++t) {
            const int l = t & 63;
            ft[t] = (l % 4) + FROW * (l / 4 % 4) + FPLANE * (l / 16);
            const int last = ft[t] + 5 * 1000 + 3 + 3 * FROW + 3 * FPLANE;
            mx = last > mx ? last : mx;
        }
        if (mx >= 2 * QN) {
            std::printf("gather pattern exceeds the LDS block: skipped\n");
        } else {
            CHECK(hipMemcpy(dtab, ft.data(), ft.size() * sizeof(int), hipMemcpyHostToDevice));
            const float ms =
                timed([&] { hipLaunchKernelGGL(k_gather, dim3(BLOCKS), dim3(256), 0, 0, dtab, out, ITERS); });
            // 6 x 16 rows x 2 paired reads = 192 instructions per iteration
            row("gather rows (ds_read2_b32, 192 per particle)", ms, (double)BLOCKS * 256 * ITERS * 192);
        }
    }
    {
        const double fops = (double)BLOCKS * 256 * ITERS * 128;
        float ms = timed([&] { hipLaunchKernelGGL(k_fma<float>, dim3(BLOCKS), dim3(256), 0, 0, out, ITERS * 8, 0.999f); });
        row("v_fma_f32 (8 chains)", ms, fops * 8);
        ms = timed([&] { hipLaunchKernelGGL(k_fma<double>, dim3(BLOCKS), dim3(256), 0, 0, out, ITERS * 8, 0.999); });
        row("v_fma_f64 (8 chains)", ms, fops * 8);
        ms = timed([&] { hipLaunchKernelGGL(k_dpp_add, dim3(BLOCKS), dim3(256), 0, 0, out, ITERS * 8, 0.5f); });
        row("v_mov_b32_dpp row_shr:1 + v_fmac_f32 pair (8 chains)", ms, fops * 8);
    }

    {
        // One 4x4x4 tile with Poisson(32) particles per cell.  Orders of its particles:
        //   cell rounds:   round r holds one particle of every cell with more than r (cell order)
        //   column rounds: round j holds one particle of every (x, y) column (4 cells stacked in
        //                  z) with more than j, a column's particles taken cell by cell in z
        //   full:          32 particles in every cell, cell rounds (every round full)
        std::mt19937 prng(4575);
        std::poisson_distribution<int> pois(32.0);
        int cnt[64];
        for (int c = 0; c < 64; ++c) cnt[c] = pois(prng);
        // sequences of (cell, round) in the flat order
        auto cell_rounds = [&](const int* cn) {
            std::vector<std::pair<int, int>> seq;
            int mx = 0;
            for (int c = 0; c < 64; ++c) mx = cn[c] > mx ? cn[c] : mx;
            for (int r = 0; r < mx; ++r)
                for (int c = 0; c < 64; ++c)
                    if (cn[c] > r) seq.push_back({c, r});
            return seq;
        };
        auto column_rounds = [&](const int* cn) {
            std::vector<int> col[16];
            for (int z = 0; z < 4; ++z)
                for (int y = 0; y < 4; ++y)
                    for (int x = 0; x < 4; ++x)
                        for (int k = 0; k < cn[x + 4 * y + 16 * z]; ++k) col[x + 4 * y].push_back(x + 4 * y + 16 * z);
            size_t mx = 0;
            for (auto& v : col) mx = v.size() > mx ? v.size() : mx;
            std::vector<std::pair<int, int>> seq;
            for (size_t j = 0; j < mx; ++j)
                for (int c = 0; c < 16; ++c)
                    if (col[c].size() > j) seq.push_back({col[c][j], (int)j});
            return seq;
        };
        int full[64];
        for (int c = 0; c < 64; ++c) full[c] = 32;
        struct Pat {
            const char* name;
            std::vector<std::pair<int, int>> seq;
        };
        // the same order with every 64-slot chunk permuted class-major: a cell's class is its
        // (x, y) place (16 classes, the bank pair of its window); the chunk's cells are sorted by
        // (index among the chunk's cells of the same class, class), so that each group of 16
        // lanes holds distinct classes where the chunk allows it (full rounds are unchanged)
        auto class_major = [&](std::vector<std::pair<int, int>> seq) {
            for (size_t b = 0; b + 64 <= seq.size(); b += 64) {
                std::vector<std::pair<int, std::pair<int, int>>> key;
                int seen[16] = {0};
                for (int l = 0; l < 64; ++l) {
                    const int c = seq[b + l].first, cls = c % 16;
                    key.push_back({seen[cls]++ * 16 + cls, seq[b + l]});
                }
                std::stable_sort(key.begin(), key.end(),
                                 [](const auto& x, const auto& y) { return x.first < y.first; });
                for (int l = 0; l < 64; ++l) seq[b + l] = key[l].second;
            }
            return seq;
        };
        std::vector<Pat> pats = {{"cell rounds, Poisson(32) tile", cell_rounds(cnt)},
                                 {"cell rounds class-major, Poisson(32) tile", class_major(cell_rounds(cnt))},
                                 {"column rounds, Poisson(32) tile", column_rounds(cnt)},
                                 {"cell rounds, 32 in every cell", cell_rounds(full)}};
        int* dchunks = nullptr;
        CHECK(hipMalloc(&dchunks, 64 * 200 * sizeof(int)));
        for (const auto& pt : pats) {
            const int nchunks = (int)(pt.seq.size() / 64);  // the last incomplete chunk is left out
            if (nchunks < 1 || nchunks > 200) continue;
            struct Layout {
                const char* what;
                bool dep;
                int row, plane, copies, copy_stride;
            };
            for (const Layout& L : {Layout{"deposit, rows 12, planes 128", true, 12, 128, 1, 0},
                                    Layout{"deposit, rows 12, planes 144", true, 12, 144, 1, 0},
                                    Layout{"deposit, rows 12, planes 136", true, 12, 136, 1, 0},
                                    Layout{"deposit, rows 8, planes 64", true, 8, 64, 1, 0},
                                    Layout{"deposit, rows 12, planes 128, 2 copies by round", true, 12, 128, 2, 1024},
                                    Layout{"deposit, rows 8, planes 64, 2 copies by round", true, 8, 64, 2, 512},
                                    Layout{"deposit, rows 8, planes 64, 3 copies by round", true, 8, 64, 3, 512},
                                    Layout{"gather, rows 10, planes 90", false, 10, 90, 1, 0}}) {
                std::vector<int> t((size_t)nchunks * 64);
                int mx = 0;
                for (int i = 0; i < nchunks * 64; ++i) {
                    const int c = pt.seq[i].first, r = pt.seq[i].second;
                    t[i] = (c % 4) + L.row * (c / 4 % 4) + L.plane * (c / 16) + (r % L.copies) * L.copy_stride;
                    const int last = L.dep ? t[i] + 3 + 4 * L.row + 4 * L.plane : t[i] + 5 * 1600 + 3 + 3 * L.row + 3 * L.plane;
                    mx = last > mx ? last : mx;
                }
                if (mx >= (L.dep ? QN : 2 * QN)) {
                    std::printf("%s: pattern exceeds the LDS block, skipped\n", L.what);
                    continue;
                }
                CHECK(hipMemcpy(dchunks, t.data(), t.size() * sizeof(int), hipMemcpyHostToDevice));
                float ms;
                double ops;
                if (L.dep) {
                    ms = timed([&] {
                        hipLaunchKernelGGL(k_chunk_deposit, dim3(BLOCKS), dim3(256), 0, 0, dchunks, nchunks, out, ITERS,
                                           L.row, L.plane);
                    });
                    ops = lane_ops;
                } else {
                    ms = timed([&] {
                        hipLaunchKernelGGL(k_chunk_gather, dim3(BLOCKS), dim3(256), 0, 0, dchunks, nchunks, out, ITERS,
                                           L.row, L.plane);
                    });
                    ops = (double)BLOCKS * 256 * ITERS * 192;
                }
                char name[120];
                std::snprintf(name, sizeof name, "%s: %s", pt.name, L.what);
                row(name, ms, ops);
            }
        }
        (void)hipFree(dchunks);
    }
    CHECK(hipDeviceSynchronize());
    CHECK(hipGetLastError());
    std::printf("status ok\n");
    (void)hipFree(out);
    (void)hipFree(dtab);
    return 0;
}
