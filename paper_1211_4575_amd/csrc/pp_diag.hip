// FP64 diagnostics: kinetic energy and momentum per species, field energies, the charge
// density (eq. "rho2", same weights as the gather), the Gauss-law residual with the
// field-order divergence, the discrete continuity residual (eq. "cc1") and div B.
//
// Charge density of the split form, once the particles are stored tile by tile: one
// workgroup per tile adds the (O+1)^3 contributions q w W of each of its particles to an LDS
// block of the tile plus its support halo (1 node below, O above), in 64-bit fixed point
// (the contribution scaled by 2^e and rounded by one fused multiply-add with 1.5*2^52, whose
// bit pattern is added with an integer atomic; the node sum is the sign-extended low 51
// bits).  The block is then added to a global 64-bit accumulator, and a last pass writes
// rho = sum * 2^-e.  A particle found outside the tile it is stored with (after a push, before
// the sort) adds its rounded contributions straight to the global accumulator.  The result
// is the exact sum of the rounded contributions, whatever the order.  The FP64 form, and a
// split species never sorted, use one thread per particle with FP64 global atomics.
#include "pp_device.hpp"
#include "pp_internal.hpp"

namespace pp {

// accumulator slots (doubles) in r->dacc
enum {
    ACC_KIN = 0,                           // [PP_MAX_SPECIES]
    ACC_MOM = ACC_KIN + PP_MAX_SPECIES,    // [PP_MAX_SPECIES][3]
    ACC_UE = ACC_MOM + 3 * PP_MAX_SPECIES,
    ACC_UB,
    ACC_UEX,
    ACC_GAUSS,  // max, stored as the bits of a non-negative double
    ACC_CC,
    ACC_DIVB,
    ACC_RELAX,      // max |rhs - A B| of the last relaxation (bits of a non-negative double)
    ACC_RELAX_RHS,  // max |rhs|
    ACC_COUNT
};
// device-only slot after the copied accumulators: 2^e of the fixed-point charge density
constexpr int ACC_RHO_SCALE = ACC_COUNT;

__device__ __forceinline__ void atomic_max_nonneg(double* p, double v) {
    atomicMax((unsigned long long*)p, (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ void block_max(double v, double* dst) {
    __shared__ double sh[256];
    __syncthreads();  // the array is reused by consecutive calls
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomic_max_nonneg(dst, sh[0]);
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        p[q] = v;
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st) {
    const int bs = 256;
    int64_t g = (n + bs - 1) / bs;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)g), dim3(bs), 0, st, p, n, v);
    return hipGetLastError();
}

// kinetic energy w V m u^2/(gamma + 1) (= w V m c^2 (gamma - 1)) and momentum w V m u
template <typename T>
__global__ void __launch_bounds__(256) k_moments(const T* __restrict__ ux, const T* __restrict__ uy,
                                                 const T* __restrict__ uz, int64_t n, double ic, double wVm, double* acc_kin,
                                                 double* acc_mom) {
    double v[4] = {0, 0, 0, 0};
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        double a = (double)ux[p], b = (double)uy[p], c = (double)uz[p];
        double u2 = a * a + b * b + c * c;
        double g = sqrt(1.0 + u2 * ic * ic);
        v[0] += u2 / (g + 1.0);
        v[1] += a;
        v[2] += b;
        v[3] += c;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) v[a] *= wVm;
    __shared__ double sh[4][256];
#pragma unroll
    for (int a = 0; a < 4; ++a) sh[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
#pragma unroll
            for (int a = 0; a < 4; ++a) sh[a][threadIdx.x] += sh[a][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomic_add_f64(acc_kin, sh[0][0]);
        for (int a = 0; a < 3; ++a) atomic_add_f64(acc_mom + a, sh[a + 1][0]);
    }
}

__global__ void __launch_bounds__(256) k_field_energy(const double* __restrict__ E, const double* __restrict__ B,
                                                      int64_t nc, double hV_eps0, double hV_imu0, double* acc) {
    double v[3] = {0, 0, 0};
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nc; q += (int64_t)gridDim.x * blockDim.x) {
        double ex = E[q], ey = E[nc + q], ez = E[2 * nc + q];
        double bx = B[q], by = B[nc + q], bz = B[2 * nc + q];
        v[0] += ex * ex + ey * ey + ez * ez;
        v[1] += bx * bx + by * by + bz * bz;
        v[2] += ex * ex;
    }
    v[0] *= hV_eps0;
    v[1] *= hV_imu0;
    v[2] *= hV_eps0;
    __shared__ double sh[3][256];
#pragma unroll
    for (int a = 0; a < 3; ++a) sh[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
#pragma unroll
            for (int a = 0; a < 3; ++a) sh[a][threadIdx.x] += sh[a][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomic_add_f64(acc + 0, sh[0][0]);
        atomic_add_f64(acc + 1, sh[1][0]);
        atomic_add_f64(acc + 2, sh[2][0]);
    }
}

// rho(node) += q w W(X - node), FP64, for either particle form
template <int O, typename T>
__global__ void __launch_bounds__(256) k_deposit_rho(int nx, int ny, int nz, const int32_t* __restrict__ cell,
                                                     const T* __restrict__ px, const T* __restrict__ py,
                                                     const T* __restrict__ pz, int64_t n, double qw, double* rho,
                                                     int split) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double X[3];
    if (split) {
        int32_t c = cell[p];
        if (c < 0 || c >= nx * ny * nz) return;
        int i = c % nx, r = c / nx, j = r % ny, k = r / ny;
        X[0] = i + (double)px[p];
        X[1] = j + (double)py[p];
        X[2] = k + (double)pz[p];
    } else {
        X[0] = (double)px[p];
        X[1] = (double)py[p];
        X[2] = (double)pz[p];
    }
    double w[3][O + 1];
    int i0[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) i0[d] = weights_abs<O>(X[d], w[d]);
    const int N[3] = {nx, ny, nz};
#pragma unroll
    for (int c = 0; c <= O; ++c) {
        int k = wrap(i0[2] + c, N[2]);
#pragma unroll
        for (int b = 0; b <= O; ++b) {
            int j = wrap(i0[1] + b, N[1]);
            double wzy = qw * w[2][c] * w[1][b];
#pragma unroll
            for (int a = 0; a <= O; ++a) {
                int i = wrap(i0[0] + a, N[0]);
                atomic_add_f64(rho + (int64_t)i + (int64_t)nx * (j + (int64_t)ny * k), wzy * w[0][a]);
            }
        }
    }
}

// ---- split form: tiled fixed-point charge deposit ------------------------------------------
struct Rho32Sp {
    const int32_t* start;  // tile starts of the stored order (ntiles + 1)
    const int32_t* cell;
    const float* pos[3];
    double qw;
};

// A workgroup deposits the particles stored in its tile's range; under a pending sort
// order that range holds the particles of the tile before their last push, which may have
// moved up to RHO_HALO cells out of it, so the LDS block covers that many cells around the
// tile (particles further away, only in flagged states, take global atomics).
constexpr int RHO_HALO = 2;

struct Rho32Args {
    int n[3], t[3], nt[3];
    int ext[3];   // LDS block extent per axis: t + 2 RHO_HALO + O + 1 (1 on a single-cell axis)
    int lo[3];    // nodes below the tile: RHO_HALO + 1 (0 on a single-cell axis)
    int halo[3];  // cells around the tile deposited in the block: RHO_HALO (0 on a single-cell axis)
    int64_t nc;
    int nsp;
    Rho32Sp sp[PP_MAX_SPECIES];
    unsigned long long* acc;  // nc, zero on entry
    const double* scale;      // 2^e
};

constexpr double RHO_MAGIC = 6755399441055744.0;  // 1.5 * 2^52
constexpr unsigned long long RHO_LOW51 = (1ull << 51) - 1ull;
constexpr long long RHO_BIT50 = 1ll << 50;

// sum of the rounded values held in the low 51 bits of a sum of bit patterns
__device__ __forceinline__ long long rho_fixed_sum(unsigned long long v) {
    return (long long)((v & RHO_LOW51) ^ (unsigned long long)RHO_BIT50) - RHO_BIT50;
}

// bit pattern of 1.5*2^52 + round(x), |x| < 2^50
__device__ __forceinline__ unsigned long long rho_pattern(double a, double b) {
    return (unsigned long long)__double_as_longlong(fma(a, b, RHO_MAGIC));
}

// 2^e with e = e0 - ceil(log2(N)) - margin, N the sum of the largest tile populations of
// the deposited species: a contribution is at most 2^(50 - ceil log2 N) and an LDS node sum
// at most 2^50 in magnitude.  margin = 1 under a pending sort order, whose tile ranges are
// the previous step's (their populations differ from the new ones by the particles that
// changed tile).
__global__ void k_rho_scale(const int32_t* __restrict__ tile_max, unsigned mask, int e0, int margin, double* scale) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    long long nb = 0;
    for (int s = 0; s < PP_MAX_SPECIES; ++s)
        if (mask & (1u << s)) nb += tile_max[s];
    int lg = 0;
    while ((1ll << lg) < nb) ++lg;
    *scale = ldexp(1.0, e0 - lg - margin);
}

template <int O>
__global__ void __launch_bounds__(256) k_rho32(Rho32Args A) {
    extern __shared__ unsigned long long rho_blk[];
    const int64_t tile = blockIdx.x;
    const int ti = (int)(tile % A.nt[0]);
    const int tj = (int)((tile / A.nt[0]) % A.nt[1]);
    const int tk = (int)(tile / ((int64_t)A.nt[0] * A.nt[1]));
    const int org[3] = {ti * A.t[0], tj * A.t[1], tk * A.t[2]};
    const int vol = A.ext[0] * A.ext[1] * A.ext[2];
    for (int q = threadIdx.x; q < vol; q += blockDim.x) rho_blk[q] = 0ull;
    __syncthreads();
    const double sc = *A.scale;
    const float flo = O == 2 ? -0.5f : 0.0f;
    const int nxy = A.n[0] * A.n[1];
    for (int s = 0; s < A.nsp; ++s) {
        const Rho32Sp& S = A.sp[s];
        const double v = S.qw * sc;
        const int32_t end = S.start[tile + 1];
        for (int32_t p = S.start[tile] + threadIdx.x; p < end; p += blockDim.x) {
            const int32_t cell = S.cell[p];
            if (cell < 0 || (int64_t)cell >= A.nc) continue;  // reported by the error flags
            const int g[3] = {cell % A.n[0], (cell / A.n[0]) % A.n[1], cell / nxy};
            const float f[3] = {S.pos[0][p], S.pos[1][p], S.pos[2][p]};
            bool finite = true, in_block = true;
            int ll[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                finite = finite && fabsf(f[d]) <= 1048576.0f;  // false for NaN and Inf as well
                int l = g[d] - org[d];  // cell relative to the tile, nearest periodic image
                if (l >= A.t[d] + A.halo[d])
                    l -= A.n[d];
                else if (l < -A.halo[d])
                    l += A.n[d];
                ll[d] = l;
                in_block = in_block && l >= -A.halo[d] && l < A.t[d] + A.halo[d] && f[d] >= flo && f[d] < flo + 2.0f;
            }
            if (!finite) continue;  // reported by the error flags
            double w[3][O + 1];
            int i0[3];
            if (in_block) {
                // support inside the block: nodes of cells -halo .. t + halo - 1 around the tile,
                // i.e. block indices 0 .. t + 2 halo + O
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    i0[d] = weights_abs<O>((double)(ll[d] + A.lo[d]) + (double)f[d], w[d]);
#pragma unroll
                for (int c = 0; c <= O; ++c) {
                    const int zc = A.ext[2] == 1 ? 0 : i0[2] + c;
#pragma unroll
                    for (int b = 0; b <= O; ++b) {
                        const int yb = A.ext[1] == 1 ? 0 : i0[1] + b;
                        const double vzy = v * w[2][c] * w[1][b];
                        const int row = A.ext[0] * (yb + A.ext[1] * zc);
#pragma unroll
                        for (int a = 0; a <= O; ++a) {
                            const int xa = A.ext[0] == 1 ? 0 : i0[0] + a;
                            atomicAdd(&rho_blk[row + xa], rho_pattern(vzy, w[0][a]));
                        }
                    }
                }
            } else {
#pragma unroll
                for (int d = 0; d < 3; ++d) i0[d] = weights_abs<O>((double)g[d] + (double)f[d], w[d]);
#pragma unroll
                for (int c = 0; c <= O; ++c) {
                    const int k = wrap(i0[2] + c, A.n[2]);
#pragma unroll
                    for (int b = 0; b <= O; ++b) {
                        const int j = wrap(i0[1] + b, A.n[1]);
                        const double vzy = v * w[2][c] * w[1][b];
#pragma unroll
                        for (int a = 0; a <= O; ++a) {
                            const int i = wrap(i0[0] + a, A.n[0]);
                            const long long x = rho_fixed_sum(rho_pattern(vzy, w[0][a]));
                            atomicAdd(A.acc + (int64_t)i + (int64_t)A.n[0] * (j + (int64_t)A.n[1] * k),
                                      (unsigned long long)x);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < vol; q += blockDim.x) {
        const long long x = rho_fixed_sum(rho_blk[q]);
        if (x == 0) continue;
        const int a = q % A.ext[0];
        const int b = (q / A.ext[0]) % A.ext[1];
        const int c = q / (A.ext[0] * A.ext[1]);
        const int i = wrap(org[0] - A.lo[0] + a, A.n[0]);
        const int j = wrap(org[1] - A.lo[1] + b, A.n[1]);
        const int k = wrap(org[2] - A.lo[2] + c, A.n[2]);
        atomicAdd(A.acc + (int64_t)i + (int64_t)A.n[0] * (j + (int64_t)A.n[1] * k), (unsigned long long)x);
    }
}

__global__ void __launch_bounds__(256) k_rho_from_fixed(const unsigned long long* __restrict__ acc, int64_t nc,
                                                        const double* __restrict__ scale, double* rho) {
    const double inv = 1.0 / *scale;  // exact: a power of two
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nc; q += (int64_t)gridDim.x * blockDim.x)
        rho[q] = (double)(long long)acc[q] * inv;
}

struct DivGeom {
    int n[3];
    int64_t nc;
    int M;
    double a[3][3];  // a_m / d
};

__device__ __forceinline__ int nbw(int i, int o, int n) {
    int j = i + o;
    while (j < 0) j += n;
    while (j >= n) j -= n;
    return j;
}

// down divergence of a face field at cell centre (i,j,k)
__device__ __forceinline__ double div_dn(const DivGeom& G, const double* F, int i, int j, int k) {
    const int c[3] = {i, j, k};
    double s = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
        const double* f = F + ax * G.nc;
        for (int m = 1; m <= G.M; ++m) {
            int hi[3] = {i, j, k}, lo[3] = {i, j, k};
            hi[ax] = nbw(c[ax], m - 1, G.n[ax]);
            lo[ax] = nbw(c[ax], -m, G.n[ax]);
            s += G.a[ax][m - 1] * (f[hi[0] + (int64_t)G.n[0] * (hi[1] + (int64_t)G.n[1] * hi[2])] -
                                   f[lo[0] + (int64_t)G.n[0] * (lo[1] + (int64_t)G.n[1] * lo[2])]);
        }
    }
    return s;
}

__device__ __forceinline__ double div_up(const DivGeom& G, const double* F, int i, int j, int k) {
    const int c[3] = {i, j, k};
    double s = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
        const double* f = F + ax * G.nc;
        for (int m = 1; m <= G.M; ++m) {
            int hi[3] = {i, j, k}, lo[3] = {i, j, k};
            hi[ax] = nbw(c[ax], m, G.n[ax]);
            lo[ax] = nbw(c[ax], -m + 1, G.n[ax]);
            s += G.a[ax][m - 1] * (f[hi[0] + (int64_t)G.n[0] * (hi[1] + (int64_t)G.n[1] * hi[2])] -
                                   f[lo[0] + (int64_t)G.n[0] * (lo[1] + (int64_t)G.n[1] * lo[2])]);
        }
    }
    return s;
}

// Gauss residual |div E - (rho + rho_bg)/eps0| and continuity residual
// |rho - rho_prev + dt div J|, max norms
__global__ void __launch_bounds__(256) k_residuals(DivGeom G, const double* __restrict__ E, const double* __restrict__ J,
                                                   const double* __restrict__ B, const double* __restrict__ rho,
                                                   const double* __restrict__ rho_prev, double rho_bg, double ieps0,
                                                   double dt, int want_rho, int have_prev, int want_divb, double* acc) {
    double g = 0.0, cc = 0.0, db = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < G.nc; q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q % G.n[0]);
        const int j = (int)((q / G.n[0]) % G.n[1]);
        const int k = (int)(q / ((int64_t)G.n[0] * G.n[1]));
        if (want_rho) {
            g = fmax(g, fabs(div_dn(G, E, i, j, k) - (rho[q] + rho_bg) * ieps0));
            if (have_prev) cc = fmax(cc, fabs(rho[q] - rho_prev[q] + dt * div_dn(G, J, i, j, k)));
        }
        if (want_divb) db = fmax(db, fabs(div_up(G, B, i, j, k)));
    }
    block_max(g, acc + 0);
    block_max(cc, acc + 1);
    block_max(db, acc + 2);
}

static void fd_coeffs(int order, double a[3]) {
    a[0] = a[1] = a[2] = 0.0;
    if (order == 2) {
        a[0] = 1.0;
    } else if (order == 4) {
        a[0] = 9.0 / 8.0;
        a[1] = -1.0 / 24.0;
    } else {
        a[0] = 75.0 / 64.0;
        a[1] = -25.0 / 384.0;
        a[2] = 3.0 / 640.0;
    }
}

template <typename T>
static void deposit_rho_species(pp_run* r, const Species& S) {
    const int bs = 256;
    const unsigned g = (unsigned)((S.n + bs - 1) / bs);
    const int split = r->p.precision == PP_PREC_FP32_SPLIT;
    const double qw = S.q * S.w;
    if (r->p.shape_order == 2)
        hipLaunchKernelGGL((k_deposit_rho<2, T>), dim3(g), dim3(bs), 0, r->stream, r->p.n[0], r->p.n[1], r->p.n[2],
                           (const int32_t*)S.cur.cell, (const T*)S.cur.pos[0], (const T*)S.cur.pos[1],
                           (const T*)S.cur.pos[2], S.n, qw, r->rho, split);
    else
        hipLaunchKernelGGL((k_deposit_rho<3, T>), dim3(g), dim3(bs), 0, r->stream, r->p.n[0], r->p.n[1], r->p.n[2],
                           (const int32_t*)S.cur.cell, (const T*)S.cur.pos[0], (const T*)S.cur.pos[1],
                           (const T*)S.cur.pos[2], S.n, qw, r->rho, split);
}

// Tiled charge deposit of the split species in mask (each stored tile by tile); writes rho.
static hipError_t launch_rho32(pp_run* r, unsigned mask) {
    Rho32Args A;
    const int O = r->p.shape_order;
    double qwmax = 0.0;
    bool pending = false;
    A.nsp = 0;
    for (int s = 0; s < PP_MAX_SPECIES; ++s) {
        if (!(mask & (1u << s))) continue;
        const Species& S = r->sp[s];
        Rho32Sp& D = A.sp[A.nsp++];
        // with a sort order pending, the buffers still follow the previous tile starts
        D.start = S.pending ? S.offsets_next : S.offsets;
        pending = pending || S.pending;
        D.cell = (const int32_t*)S.cur.cell;
        for (int d = 0; d < 3; ++d) D.pos[d] = (const float*)S.cur.pos[d];
        D.qw = S.q * S.w;
        qwmax = fabs(D.qw) > qwmax ? fabs(D.qw) : qwmax;
    }
    int vol = 1;
    for (int d = 0; d < 3; ++d) {
        A.n[d] = r->p.n[d];
        A.t[d] = r->g.t[d];
        A.nt[d] = r->g.nt[d];
        const bool single = r->p.n[d] == 1;
        A.ext[d] = single ? 1 : r->g.t[d] + 2 * RHO_HALO + O + 1;
        A.lo[d] = single ? 0 : RHO_HALO + 1;
        A.halo[d] = single ? 0 : RHO_HALO;
        vol *= A.ext[d];
    }
    A.nc = r->g.ncell;
    A.acc = (unsigned long long*)r->Jq;  // free between steps: the particle kernel clears it
    A.scale = r->dacc + ACC_RHO_SCALE;
    // every contribution is at most |q w| (the weights of a node are at most 1)
    int e0 = 50 - (int)ceil(log2(qwmax));
    if (e0 > 1000) e0 = 1000;
    hipLaunchKernelGGL(k_rho_scale, dim3(1), dim3(64), 0, r->stream, (const int32_t*)r->tile_max, mask, e0,
                       pending ? 1 : 0, r->dacc + ACC_RHO_SCALE);
    hipError_t e = launch_fill((double*)r->Jq, A.nc, 0.0, r->stream);  // all-zero bits
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)vol * sizeof(unsigned long long);
    if (O == 2)
        hipLaunchKernelGGL(k_rho32<2>, dim3((unsigned)r->g.ntiles), dim3(256), lds, r->stream, A);
    else
        hipLaunchKernelGGL(k_rho32<3>, dim3((unsigned)r->g.ntiles), dim3(256), lds, r->stream, A);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t g = (A.nc + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_rho_from_fixed, dim3((unsigned)g), dim3(256), 0, r->stream,
                       (const unsigned long long*)r->Jq, A.nc, (const double*)(r->dacc + ACC_RHO_SCALE), r->rho);
    return hipGetLastError();
}

// rho of the current particle positions into r->rho.  Split species stored tile by tile
// (sorted, or pushed since the last sort) go through the tiled fixed-point deposit, which
// writes every node of rho; the others are added with FP64 atomics.
hipError_t deposit_rho_all(pp_run* r) {
    const int64_t nc = r->g.ncell;
    const bool split = r->p.precision == PP_PREC_FP32_SPLIT;
    unsigned tiled = 0;
    if (split)
        for (int s = 0; s < PP_MAX_SPECIES; ++s) {
            const Species& S = r->sp[s];
            if (S.active && S.n > 0 && S.q * S.w != 0.0 && (S.sorted || S.ranked)) tiled |= 1u << s;
        }
    hipError_t e = tiled ? launch_rho32(r, tiled) : launch_fill(r->rho, nc, 0.0, r->stream);
    if (e != hipSuccess) return e;
    for (int s = 0; s < PP_MAX_SPECIES; ++s) {
        const Species& S = r->sp[s];
        if (!S.active || S.n == 0 || S.q * S.w == 0.0 || (tiled & (1u << s))) continue;
        if (split)
            deposit_rho_species<float>(r, S);
        else
            deposit_rho_species<double>(r, S);
    }
    return hipGetLastError();
}

// Fills host_out[0..ACC_COUNT) with the accumulators and [ACC_COUNT] with the flag word.
hipError_t launch_diag(pp_run* r, uint32_t what, double* host_out) {
    const int bs = 256;
    const int64_t nc = r->g.ncell;
    // a pending sort order needs no move here: the moments are sums over every particle and
    // the charge deposit follows the tile starts of the buffers as they are
    hipError_t e = launch_fill(r->dacc, ACC_COUNT, 0.0, r->stream);
    if (e != hipSuccess) return e;
    const bool split = r->p.precision == PP_PREC_FP32_SPLIT;
    const double V = r->p.d[0] * r->p.d[1] * r->p.d[2];
    const double ic = 1.0 / r->p.c;
    if (what & PP_DIAG_MOMENTS) {
        for (int s = 0; s < PP_MAX_SPECIES; ++s) {
            const Species& S = r->sp[s];
            if (!S.active || S.n == 0) continue;
            int64_t g = (S.n + bs - 1) / bs;
            if (g > 4096) g = 4096;
            const double wVm = S.w * V * S.m;
            if (split)
                hipLaunchKernelGGL(k_moments<float>, dim3((unsigned)g), dim3(bs), 0, r->stream, (const float*)S.cur.u[0],
                                   (const float*)S.cur.u[1], (const float*)S.cur.u[2], S.n, ic, wVm, r->dacc + ACC_KIN + s,
                                   r->dacc + ACC_MOM + 3 * s);
            else
                hipLaunchKernelGGL(k_moments<double>, dim3((unsigned)g), dim3(bs), 0, r->stream,
                                   (const double*)S.cur.u[0], (const double*)S.cur.u[1], (const double*)S.cur.u[2], S.n,
                                   ic, wVm, r->dacc + ACC_KIN + s, r->dacc + ACC_MOM + 3 * s);
        }
    }
    if (what & PP_DIAG_FIELDS) {
        int64_t g = (nc + bs - 1) / bs;
        if (g > 4096) g = 4096;
        const double mu0 = 1.0 / (r->p.eps0 * r->p.c * r->p.c);
        hipLaunchKernelGGL(k_field_energy, dim3((unsigned)g), dim3(bs), 0, r->stream, (const double*)r->mesh.E,
                           (const double*)r->mesh.B, nc, 0.5 * r->p.eps0 * V, 0.5 * V / mu0, r->dacc + ACC_UE);
    }
    const bool want_rho = (what & PP_DIAG_RHO) != 0;
    const bool want_divb = (what & PP_DIAG_DIVB) != 0;
    bool have_prev = false;
    if (want_rho) {
        e = deposit_rho_all(r);
        if (e != hipSuccess) return e;
        have_prev = r->rho_prev_step >= 0 && r->rho_prev_step == r->step - 1;
    }
    if (want_rho || want_divb) {
        DivGeom G;
        for (int d = 0; d < 3; ++d) G.n[d] = r->p.n[d];
        G.nc = nc;
        G.M = r->p.field_order / 2;
        double a[3];
        fd_coeffs(r->p.field_order, a);
        for (int d = 0; d < 3; ++d)
            for (int m = 0; m < 3; ++m) G.a[d][m] = a[m] / r->p.d[d];
        int64_t g = (nc + bs - 1) / bs;
        if (g > 4096) g = 4096;
        hipLaunchKernelGGL(k_residuals, dim3((unsigned)g), dim3(bs), 0, r->stream, G, (const double*)r->mesh.E,
                           (const double*)r->mesh.J, (const double*)r->mesh.B, (const double*)r->rho,
                           (const double*)r->rho_prev, r->p.rho_background, 1.0 / r->p.eps0, r->dt_drift, want_rho ? 1 : 0,
                           have_prev ? 1 : 0, want_divb ? 1 : 0, r->dacc + ACC_GAUSS);
    }
    const bool want_relax = (what & PP_DIAG_RELAX) != 0 && r->rhs_valid;
    if (want_relax) {
        e = launch_relax_resid(r, r->dacc + ACC_RELAX);
        if (e != hipSuccess) return e;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(host_out, r->dacc, ACC_COUNT * sizeof(double), hipMemcpyDeviceToHost, r->stream);
    if (e != hipSuccess) return e;
    int32_t flags = 0;
    e = hipMemcpyAsync(&flags, r->flags, sizeof(int32_t), hipMemcpyDeviceToHost, r->stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return e;
    host_out[ACC_COUNT] = (double)flags;
    host_out[ACC_COUNT + 1] = have_prev ? 1.0 : 0.0;
    host_out[ACC_COUNT + 2] = want_relax ? 1.0 : 0.0;
    // clear the flags and keep rho for the next continuity check
    e = hipMemsetAsync(r->flags, 0, sizeof(int32_t), r->stream);
    if (e != hipSuccess) return e;
    if (want_rho) {
        double* t = r->rho_prev;
        r->rho_prev = r->rho;
        r->rho = t;
        r->rho_prev_step = r->step;
    }
    return hipSuccess;
}

int diag_acc_count() { return ACC_COUNT; }

}  // namespace pp
