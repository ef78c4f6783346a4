// On-device twin of the host particle loaders (inputs.py): input generation only.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/pp_inputs.h"

namespace {

struct U4 {
    uint32_t x, y, z, w;
};

// Philox-4x32-R block function (Salmon, Moraes, Dror & Shaw 2011): R rounds of two 32x32->64
// multiplies, key bumped by the Weyl constants between rounds.
__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t p0 = (uint64_t)M0 * c.x;
        const uint64_t p1 = (uint64_t)M1 * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    }
    return c;
}

__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    const double hi = (double)(a >> 5), lo = (double)(b >> 6);
    return (hi * 67108864.0 + lo + 0.5) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ void uniform_pair(uint64_t seed, uint64_t idx, uint32_t blk, uint32_t stream, double& a,
                                             double& b) {
    U4 r = philox10(U4{(uint32_t)idx, (uint32_t)(idx >> 32), blk, stream}, (uint32_t)seed, (uint32_t)(seed >> 32));
    a = u53(r.x, r.y);
    b = u53(r.z, r.w);
}

__device__ __forceinline__ uint32_t stream_id(int wl, int sp, int purpose) {
    return (uint32_t)((wl << 8) | (sp << 4) | purpose);
}

// Split form of positions X[3] in [0, n): mode 1 = nearest node (offset in [-1/2, 1/2)),
// mode 2 = node below (offset in [0, 1)); the offset is rounded to float and a particle whose
// rounded offset lands on the upper end of the range moves to the next cell.
__device__ __forceinline__ int32_t to_split(const double* X, const int* n, int mode, float* off) {
    const double lo = mode == 1 ? -0.5 : 0.0;
    int64_t ijk[3];
    for (int d = 0; d < 3; ++d) {
        double c = floor(X[d] - lo);
        float o = (float)(X[d] - c);
        if (o >= (float)(lo + 1.0)) {  // the moved particle starts the next cell's range
            c += 1.0;
            o = fmaxf((float)(X[d] - c), (float)lo);
        }
        off[d] = o;
        int64_t ci = (int64_t)c % n[d];
        ijk[d] = ci < 0 ? ci + n[d] : ci;
    }
    return (int32_t)(ijk[0] + (int64_t)n[0] * (ijk[1] + (int64_t)n[1] * ijk[2]));
}

__global__ void k_philox_blocks(uint64_t seed, uint32_t block, uint32_t stream, int64_t ctr0, int64_t count,
                                uint32_t* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint64_t c = (uint64_t)(i + ctr0);
    U4 r = philox10(U4{(uint32_t)c, (uint32_t)(c >> 32), block, stream}, (uint32_t)seed, (uint32_t)(seed >> 32));
    out[4 * i + 0] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
}

struct MJArgs {
    uint64_t seed;
    int n[3];
    int64_t start, count;
    double theta;
    int split;
    int32_t* cell[2];
    void* off[2][3];
    void* u[2][3];
};

__global__ void __launch_bounds__(256) k_pair_mj(MJArgs A) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= A.count) return;
    const uint64_t idx = (uint64_t)(A.start + l);
    double U[4];
    uniform_pair(A.seed, idx, 0, stream_id(3, 0, 0), U[0], U[1]);
    uniform_pair(A.seed, idx, 1, stream_id(3, 0, 0), U[2], U[3]);
    double pos[3];
    for (int d = 0; d < 3; ++d) {
        double x = U[d] * A.n[d];
        pos[d] = x >= A.n[d] ? 0.0 : x;
    }
    int32_t cellv = 0;
    float offf[3];
    if (A.split) cellv = to_split(pos, A.n, A.split, offf);
    for (int s = 0; s < 2; ++s) {
        // Sobol rejection: attempt t uses draw blocks 2t, 2t+1
        double mag = 0.0;
        for (int t = 0; t < 64; ++t) {
            double x1, x2, x3, x4;
            uniform_pair(A.seed, idx, 2 * t, stream_id(3, s, 1), x1, x2);
            uniform_pair(A.seed, idx, 2 * t + 1, stream_id(3, s, 1), x3, x4);
            const double uu = -A.theta * log(x1 * x2 * x3);
            const double eta = -A.theta * log(x1 * x2 * x3 * x4);
            if (eta * eta - uu * uu > 1.0) {
                mag = uu;
                break;
            }
        }
        double a, b;
        uniform_pair(A.seed, idx, 0, stream_id(3, s, 2), a, b);
        const double cz = 2.0 * a - 1.0;
        const double ph = 2.0 * M_PI * b;
        const double sz = sqrt(fmax(0.0, 1.0 - cz * cz));
        const double uv[3] = {sz * cos(ph) * mag, sz * sin(ph) * mag, cz * mag};
        if (A.split) {
            A.cell[s][l] = cellv;
            for (int d = 0; d < 3; ++d) {
                ((float*)A.off[s][d])[l] = offf[d];
                ((float*)A.u[s][d])[l] = (float)uv[d];
            }
        } else {
            for (int d = 0; d < 3; ++d) {
                ((double*)A.off[s][d])[l] = pos[d];
                ((double*)A.u[s][d])[l] = uv[d];
            }
        }
    }
}

struct TSArgs {
    uint64_t seed;
    int wl;
    int n[3], k[3];
    int64_t npart;
    double drift[2];
    double uth;
    int split;
    int32_t* cell[2];
    void* off[2][3];
    void* u[2][3];
};

// Two beams on a quiet lattice: particle p sits at lattice point (ix, iy, iz), x fastest, of
// k[d] points per cell per axis at offsets (a + 1/2)/k; both beams share the points.  Proper
// velocity = drift along x + uth * standard normals (Box-Muller of draw blocks 0 and 1).
__global__ void __launch_bounds__(256) k_two_stream(TSArgs A) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.npart) return;
    const int64_t Lx = (int64_t)A.n[0] * A.k[0], Ly = (int64_t)A.n[1] * A.k[1];
    const int64_t ix = p % Lx, iy = (p / Lx) % Ly, iz = p / (Lx * Ly);
    const double X[3] = {((double)ix + 0.5) / A.k[0], ((double)iy + 0.5) / A.k[1], ((double)iz + 0.5) / A.k[2]};
    int32_t cellv = 0;
    float offf[3];
    if (A.split) cellv = to_split(X, A.n, A.split, offf);
    for (int s = 0; s < 2; ++s) {
        double U[4];
        uniform_pair(A.seed, (uint64_t)p, 0, stream_id(A.wl, s, 1), U[0], U[1]);
        uniform_pair(A.seed, (uint64_t)p, 1, stream_id(A.wl, s, 1), U[2], U[3]);
        const double r0 = sqrt(-2.0 * log(U[0])), t0 = 2.0 * M_PI * U[1];
        const double r1 = sqrt(-2.0 * log(U[2])), t1 = 2.0 * M_PI * U[3];
        const double g[3] = {r0 * cos(t0), r0 * sin(t0), r1 * cos(t1)};
        const double uv[3] = {A.drift[s] + A.uth * g[0], A.uth * g[1], A.uth * g[2]};
        if (A.split) {
            A.cell[s][p] = cellv;
            for (int d = 0; d < 3; ++d) {
                ((float*)A.off[s][d])[p] = offf[d];
                ((float*)A.u[s][d])[p] = (float)uv[d];
            }
        } else {
            for (int d = 0; d < 3; ++d) {
                ((double*)A.off[s][d])[p] = X[d];
                ((double*)A.u[s][d])[p] = uv[d];
            }
        }
    }
}

struct KHArgs {
    uint64_t seed;
    int n[3];
    int64_t start, count;
    double v0, width, uth;
    int split;
    int32_t* cell[2];
    void* off[2][3];
    void* u[2][3];
};

// Kelvin-Helmholtz load (inputs.kelvin_helmholtz): uniform positions (stream 4/0/0, draw
// blocks 0 and 1), bulk flow vx(y) = v0 (tanh((y - Ly/4)/width) - tanh((y - 3Ly/4)/width) - 1)
// for both species at the same positions, thermal proper velocities (streams 4/s/1) plus
// gamma(vx) vx along x.
__global__ void __launch_bounds__(256) k_kelvin_helmholtz(KHArgs A) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= A.count) return;
    const uint64_t idx = (uint64_t)(A.start + l);
    double U[4];
    uniform_pair(A.seed, idx, 0, stream_id(4, 0, 0), U[0], U[1]);
    uniform_pair(A.seed, idx, 1, stream_id(4, 0, 0), U[2], U[3]);
    double pos[3];
    for (int d = 0; d < 3; ++d) {
        double x = U[d] * A.n[d];
        pos[d] = x >= A.n[d] ? 0.0 : x;
    }
    const double Ly = (double)A.n[1];
    const double vx = A.v0 * (tanh((pos[1] - Ly / 4) / A.width) - tanh((pos[1] - 3 * Ly / 4) / A.width) - 1.0);
    const double g = 1.0 / sqrt(1.0 - vx * vx);
    int32_t cellv = 0;
    float offf[3];
    if (A.split) cellv = to_split(pos, A.n, A.split, offf);
    for (int s = 0; s < 2; ++s) {
        double V[4];
        uniform_pair(A.seed, idx, 0, stream_id(4, s, 1), V[0], V[1]);
        uniform_pair(A.seed, idx, 1, stream_id(4, s, 1), V[2], V[3]);
        const double r0 = sqrt(-2.0 * log(V[0])), t0 = 2.0 * M_PI * V[1];
        const double r1 = sqrt(-2.0 * log(V[2])), t1 = 2.0 * M_PI * V[3];
        const double uv[3] = {A.uth * r0 * cos(t0) + vx * g, A.uth * r0 * sin(t0), A.uth * r1 * cos(t1)};
        if (A.split) {
            A.cell[s][l] = cellv;
            for (int d = 0; d < 3; ++d) {
                ((float*)A.off[s][d])[l] = offf[d];
                ((float*)A.u[s][d])[l] = (float)uv[d];
            }
        } else {
            for (int d = 0; d < 3; ++d) {
                ((double*)A.off[s][d])[l] = pos[d];
                ((double*)A.u[s][d])[l] = uv[d];
            }
        }
    }
}

struct MMIArgs {
    uint64_t seed;
    int n[3];
    int64_t start, count;
    double gamma_b, sig[4];  // beam Lorentz factor, thermal spread per species
    int split;
    int quiet;  // pairs 2k, 2k+1 at one position with opposite rest-frame thermal velocities
    int lat[3];  // sub-lattice points per cell and axis (0: uniform random positions)
    int32_t* cell[4];
    void* off[4][3];
    void* u[4][3];
};

// Mixed-mode two-stream load (inputs.mmi): beam positions (stream 5/0/0) shared by species 0
// and 1, background positions (stream 5/2/0) shared by species 2 and 3; Gaussian rest-frame
// proper velocities (streams 5/s/1) of spread sig[s], species 0 and 1 boosted along +z.
__global__ void __launch_bounds__(256) k_mmi(MMIArgs A) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= A.count) return;
    const uint64_t pidx = (uint64_t)(A.start + l);
    const uint64_t idx = A.quiet ? (pidx & ~1ull) : pidx;  // the index whose draws are used
    const double sgn = A.quiet && (pidx & 1ull) ? -1.0 : 1.0;
    const double beta = sqrt(1.0 - 1.0 / (A.gamma_b * A.gamma_b));
    for (int pop = 0; pop < 2; ++pop) {
        double pos[3];
        if (A.lat[0] > 0) {  // regular lattice: point pidx mod ppc of cell pidx div ppc
            const int64_t ppc = (int64_t)A.lat[0] * A.lat[1] * A.lat[2];
            const int64_t c = (int64_t)pidx / ppc, sub = (int64_t)pidx % ppc;
            const int64_t cell[3] = {c % A.n[0], (c / A.n[0]) % A.n[1], c / ((int64_t)A.n[0] * A.n[1])};
            const int64_t pt[3] = {sub % A.lat[0], (sub / A.lat[0]) % A.lat[1], sub / ((int64_t)A.lat[0] * A.lat[1])};
            for (int d = 0; d < 3; ++d) pos[d] = (double)cell[d] + ((double)pt[d] + 0.5) / (double)A.lat[d];
        } else {
            double U[4];
            uniform_pair(A.seed, idx, 0, stream_id(5, 2 * pop, 0), U[0], U[1]);
            uniform_pair(A.seed, idx, 1, stream_id(5, 2 * pop, 0), U[2], U[3]);
            for (int d = 0; d < 3; ++d) {
                const double x = U[d] * A.n[d];
                pos[d] = x >= A.n[d] ? 0.0 : x;
            }
        }
        int32_t cellv = 0;
        float offf[3];
        if (A.split) cellv = to_split(pos, A.n, A.split, offf);
        for (int h = 0; h < 2; ++h) {
            const int s = 2 * pop + h;
            double V[4];
            uniform_pair(A.seed, idx, 0, stream_id(5, s, 1), V[0], V[1]);
            uniform_pair(A.seed, idx, 1, stream_id(5, s, 1), V[2], V[3]);
            const double r0 = sqrt(-2.0 * log(V[0])), t0 = 2.0 * M_PI * V[1];
            const double r1 = sqrt(-2.0 * log(V[2])), t1 = 2.0 * M_PI * V[3];
            double uv[3] = {sgn * (A.sig[s] * r0 * cos(t0)), sgn * (A.sig[s] * r0 * sin(t0)),
                            sgn * (A.sig[s] * r1 * cos(t1))};
            if (pop == 0 && A.gamma_b != 1.0) {
                const double g = sqrt(1.0 + uv[0] * uv[0] + uv[1] * uv[1] + uv[2] * uv[2]);
                uv[2] = A.gamma_b * (uv[2] + beta * g);
            }
            if (A.split) {
                A.cell[s][l] = cellv;
                for (int d = 0; d < 3; ++d) {
                    ((float*)A.off[s][d])[l] = offf[d];
                    ((float*)A.u[s][d])[l] = (float)uv[d];
                }
            } else {
                for (int d = 0; d < 3; ++d) {
                    ((double*)A.off[s][d])[l] = pos[d];
                    ((double*)A.u[s][d])[l] = uv[d];
                }
            }
        }
    }
}

}  // namespace

extern "C" {

int ppi_two_stream_lattice(uint64_t seed, int32_t wl, const int32_t n[3], const int32_t k[3], double v_beam,
                           double uth, int32_t split, int32_t* const cell[2], void* const off[2][3],
                           void* const u[2][3], void* hip_stream) {
    if (!n || !k || !(v_beam >= 0.0 && v_beam < 1.0) || !(uth >= 0.0)) return -1;
    TSArgs A;
    A.seed = seed;
    A.wl = wl;
    A.npart = 1;
    for (int d = 0; d < 3; ++d) {
        if (n[d] < 1 || k[d] < 1) return -1;
        A.n[d] = n[d];
        A.k[d] = k[d];
        A.npart *= (int64_t)n[d] * k[d];
    }
    const double g0 = 1.0 / sqrt(1.0 - v_beam * v_beam);
    A.drift[0] = v_beam * g0;
    A.drift[1] = -v_beam * g0;
    A.uth = uth;
    if (split < 0 || split > 2) return -1;
    A.split = split;
    for (int s = 0; s < 2; ++s) {
        A.cell[s] = cell ? cell[s] : nullptr;
        if (split && !A.cell[s]) return -1;
        for (int d = 0; d < 3; ++d) {
            A.off[s][d] = off[s][d];
            A.u[s][d] = u[s][d];
            if (!A.off[s][d] || !A.u[s][d]) return -1;
        }
    }
    const int bs = 256;
    hipLaunchKernelGGL(k_two_stream, dim3((unsigned)((A.npart + bs - 1) / bs)), dim3(bs), 0, (hipStream_t)hip_stream, A);
    return hipGetLastError() == hipSuccess ? 0 : -6;
}


int ppi_philox_blocks(uint64_t seed, uint32_t block, uint32_t stream, int64_t ctr0, int64_t count, uint32_t* out,
                      void* hip_stream) {
    if (count < 0 || (count > 0 && !out)) return -1;
    if (count == 0) return 0;
    const int bs = 256;
    hipLaunchKernelGGL(k_philox_blocks, dim3((unsigned)((count + bs - 1) / bs)), dim3(bs), 0, (hipStream_t)hip_stream,
                       seed, block, stream, ctr0, count, out);
    return hipGetLastError() == hipSuccess ? 0 : -6;
}

int ppi_pair_maxwell_juttner(uint64_t seed, const int32_t n[3], int64_t start, int64_t count, double theta,
                             int32_t split, int32_t* const cell[2], void* const off[2][3], void* const u[2][3],
                             void* hip_stream) {
    if (!n || count < 0 || start < 0 || !(theta > 0.0)) return -1;
    for (int d = 0; d < 3; ++d)
        if (n[d] < 1) return -1;
    if (count == 0) return 0;
    MJArgs A;
    A.seed = seed;
    for (int d = 0; d < 3; ++d) A.n[d] = n[d];
    A.start = start;
    A.count = count;
    A.theta = theta;
    if (split < 0 || split > 2) return -1;
    A.split = split;
    for (int s = 0; s < 2; ++s) {
        A.cell[s] = cell ? cell[s] : nullptr;
        if (split && !A.cell[s]) return -1;
        for (int d = 0; d < 3; ++d) {
            A.off[s][d] = off[s][d];
            A.u[s][d] = u[s][d];
            if (!A.off[s][d] || !A.u[s][d]) return -1;
        }
    }
    const int bs = 256;
    hipLaunchKernelGGL(k_pair_mj, dim3((unsigned)((count + bs - 1) / bs)), dim3(bs), 0, (hipStream_t)hip_stream, A);
    return hipGetLastError() == hipSuccess ? 0 : -6;
}

int ppi_kelvin_helmholtz(uint64_t seed, const int32_t n[3], int64_t start, int64_t count, double v0, double width,
                         double uth, int32_t split, int32_t* const cell[2], void* const off[2][3], void* const u[2][3],
                         void* hip_stream) {
    if (!n || start < 0 || count < 0 || !(v0 >= 0.0 && v0 < 0.5) || !(width > 0.0) || !(uth >= 0.0)) return -1;
    for (int d = 0; d < 3; ++d)
        if (n[d] < 1) return -1;
    if (split < 0 || split > 2) return -1;
    if (count == 0) return 0;
    KHArgs A;
    A.seed = seed;
    for (int d = 0; d < 3; ++d) A.n[d] = n[d];
    A.start = start;
    A.count = count;
    A.v0 = v0;
    A.width = width;
    A.uth = uth;
    A.split = split;
    for (int s = 0; s < 2; ++s) {
        A.cell[s] = cell ? cell[s] : nullptr;
        if (split && !A.cell[s]) return -1;
        for (int d = 0; d < 3; ++d) {
            A.off[s][d] = off[s][d];
            A.u[s][d] = u[s][d];
            if (!A.off[s][d] || !A.u[s][d]) return -1;
        }
    }
    const int bs = 256;
    hipLaunchKernelGGL(k_kelvin_helmholtz, dim3((unsigned)((count + bs - 1) / bs)), dim3(bs), 0, (hipStream_t)hip_stream, A);
    return hipGetLastError() == hipSuccess ? 0 : -6;
}

int ppi_mmi(uint64_t seed, const int32_t n[3], int64_t start, int64_t count, double gamma_b, double T_b, double T_p,
            double mass_ratio, int32_t quiet, const int32_t lattice[3], int32_t split, int32_t* const cell[4],
            void* const off[4][3], void* const u[4][3], void* hip_stream) {
    if (!n || start < 0 || count < 0 || !(gamma_b >= 1.0) || !(T_b >= 0.0) || !(T_p >= 0.0) || !(mass_ratio > 0.0))
        return -1;
    if (lattice && (lattice[0] < 1 || lattice[1] < 1 || lattice[2] < 1)) return -1;
    for (int d = 0; d < 3; ++d)
        if (n[d] < 1) return -1;
    if (split < 0 || split > 2 || quiet < 0 || quiet > 1) return -1;
    if (count == 0) return 0;
    MMIArgs A;
    A.quiet = quiet;
    for (int d = 0; d < 3; ++d) A.lat[d] = lattice ? lattice[d] : 0;
    A.seed = seed;
    for (int d = 0; d < 3; ++d) A.n[d] = n[d];
    A.start = start;
    A.count = count;
    A.gamma_b = gamma_b;
    A.sig[0] = sqrt(T_b);
    A.sig[1] = sqrt(T_b / mass_ratio);
    A.sig[2] = sqrt(T_p);
    A.sig[3] = sqrt(T_p / mass_ratio);
    A.split = split;
    for (int s = 0; s < 4; ++s) {
        A.cell[s] = cell ? cell[s] : nullptr;
        if (split && !A.cell[s]) return -1;
        for (int d = 0; d < 3; ++d) {
            A.off[s][d] = off[s][d];
            A.u[s][d] = u[s][d];
            if (!A.off[s][d] || !A.u[s][d]) return -1;
        }
    }
    const int bs = 256;
    hipLaunchKernelGGL(k_mmi, dim3((unsigned)((count + bs - 1) / bs)), dim3(bs), 0, (hipStream_t)hip_stream, A);
    return hipGetLastError() == hipSuccess ? 0 : -6;
}

}  // extern "C"
