// Field kernels: the implicit B / explicit E step (Sec. III.B, eqs. "bnplus1",
// "enplus1", "EllipticB") and the high-order current line solve (Sec. III.C, eqs.
// "jj6d", "penta").  Mesh arrays are FP64, x fastest, periodic.
#include "pp_device.hpp"
#include "pp_internal.hpp"

namespace pp {

// Threads of a field launch: a block of 256 threads covers rows of x-consecutive cells
// (a row of nx cells, padded to a power of two, several rows per block) or, for nx > 256, a
// 256-cell chunk of one row; the remaining indices j, k come from the row number.  All
// indices are 32-bit (a box has at most 2^30 cells).
struct FieldGeom {
    int n[3];
    int64_t nc;
    int M;           // half-width of the first-derivative stencil (order / 2)
    double a[3][3];  // a[axis][m-1] / d[axis]: first-derivative coefficients
    int R;           // Laplacian half-width 2M - 1
    double L[3][11]; // Laplacian stencil per axis, offsets -R..R
    int xchunks;     // 256-cell chunks per row (nx > 256), else 1
    int xbits;       // log2 of the padded row length inside a block (<= 8)
    int rows;        // ny * nz
    int rpb;         // rows per block
    double inv_ny;   // 1 / ny (row -> j, k)
    int small;       // an axis shorter than the stencil reach: general wrap
};

constexpr int FIELD_BS = 256;

// index o cells away from i on a periodic axis of n cells
__device__ __forceinline__ int nbw(int i, int o, int n, int small) {
    int j = i + o;
    if (small) {
        j %= n;
        return j < 0 ? j + n : j;
    }
    return j < 0 ? j + n : (j >= n ? j - n : j);
}

// cell of thread t in block b of a run's launch; false for padding threads
__device__ __forceinline__ bool field_cell(const FieldGeom& G, int64_t b, int t, int& i, int& j, int& k) {
    const int xc = (int)(b % G.xchunks);
    const int64_t rb = b / G.xchunks;
    i = xc * FIELD_BS + (t & ((1 << G.xbits) - 1));
    const int64_t row = rb * G.rpb + (t >> G.xbits);
    if (i >= G.n[0] || row >= G.rows) return false;
    k = (int)floor(((double)row + 0.5) * G.inv_ny);
    j = (int)(row - (int64_t)k * G.n[1]);
    if (j < 0) {
        j += G.n[1];
        --k;
    } else if (j >= G.n[1]) {
        j -= G.n[1];
        ++k;
    }
    return true;
}

__device__ __forceinline__ int lin(const FieldGeom& G, int i, int j, int k) { return i + G.n[0] * (j + G.n[1] * k); }

// up-shifted derivative along axis ax of f (values on integer nodes along ax) at cell (i,j,k):
// sum_m a_m (f[i+m] - f[i-m+1]) / d
__device__ __forceinline__ double dup(const FieldGeom& G, const double* __restrict__ f, int ax, int i, int j, int k) {
    const int c[3] = {i, j, k};
    double s = 0.0;
    for (int m = 1; m <= G.M; ++m) {
        int hi[3] = {i, j, k}, lo[3] = {i, j, k};
        hi[ax] = nbw(c[ax], m, G.n[ax], G.small);
        lo[ax] = nbw(c[ax], -m + 1, G.n[ax], G.small);
        s += G.a[ax][m - 1] * (f[lin(G, hi[0], hi[1], hi[2])] - f[lin(G, lo[0], lo[1], lo[2])]);
    }
    return s;
}

// down-shifted derivative: sum_m a_m (g[i+m-1] - g[i-m]) / d
__device__ __forceinline__ double ddn(const FieldGeom& G, const double* __restrict__ f, int ax, int i, int j, int k) {
    const int c[3] = {i, j, k};
    double s = 0.0;
    for (int m = 1; m <= G.M; ++m) {
        int hi[3] = {i, j, k}, lo[3] = {i, j, k};
        hi[ax] = nbw(c[ax], m - 1, G.n[ax], G.small);
        lo[ax] = nbw(c[ax], -m, G.n[ax], G.small);
        s += G.a[ax][m - 1] * (f[lin(G, hi[0], hi[1], hi[2])] - f[lin(G, lo[0], lo[1], lo[2])]);
    }
    return s;
}

// composed Laplacian (d- after d+) of f at (i,j,k)
__device__ __forceinline__ double lap(const FieldGeom& G, const double* __restrict__ f, int i, int j, int k) {
    const int nx = G.n[0], nxy = G.n[0] * G.n[1];
    const int rowx = nx * (j + G.n[1] * k);
    const int colyz = i + nxy * k;
    const int colzx = i + nx * j;
    double s = 0.0;
    for (int o = -G.R; o <= G.R; ++o) {
        s += G.L[0][o + G.R] * f[rowx + nbw(i, o, nx, G.small)];
        s += G.L[1][o + G.R] * f[colyz + nx * nbw(j, o, G.n[1], G.small)];
        s += G.L[2][o + G.R] * f[colzx + nxy * nbw(k, o, G.n[2], G.small)];
    }
    return s;
}

// Everything one field step of one run needs (the single-run launches pass it by value,
// the batched launches read a table of them).
struct FieldDesc {
    FieldGeom G;
    double* E;
    double* B;
    const double* J;
    double* Bn;  // copy of B^n
    double* Bw;  // relaxation partner
    double* R;   // right-hand side
    const double* omega;        // Chebyshev weights omega_k, k = 1..sweeps (device)
    const double* rho;          // charge density (Gauss-law filter)
    double rho_bg, ieps0, kappa;  // background density, 1/eps0, filter damping
    double cab, dt, cj;         // alpha beta s, dt, alpha c^2 mu0 dt^2   (s = c^2 dt^2)
    double al2s, gdiag;         // alpha^2 s, gamma / diagonal
    double al, be, c2dt, mu0;   // alpha, beta, c^2 dt, mu0
    int sweeps;
};

__device__ __forceinline__ void copy_body(const FieldDesc& D, int q) {
#pragma unroll
    for (int c = 0; c < 3; ++c) D.Bn[c * D.G.nc + q] = D.B[c * D.G.nc + q];
}

// rhs = B + alpha beta s lap B - dt curl+ E + alpha c^2 mu0 dt^2 curl+ J   (B = B^n from Bn)
__device__ __forceinline__ void rhs_body(const FieldDesc& D, int i, int j, int k) {
    const FieldGeom& G = D.G;
    const int q = lin(G, i, j, k);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int d1 = (c + 1) % 3, d2 = (c + 2) % 3;
        const double* Bc = D.Bn + c * G.nc;
        double curlE = dup(G, D.E + d2 * G.nc, d1, i, j, k) - dup(G, D.E + d1 * G.nc, d2, i, j, k);
        double curlJ = dup(G, D.J + d2 * G.nc, d1, i, j, k) - dup(G, D.J + d1 * G.nc, d2, i, j, k);
        D.R[c * G.nc + q] = Bc[q] + D.cab * lap(G, Bc, i, j, k) - D.dt * curlE + D.cj * curlJ;
    }
}

// Sweep k (1-based) of the Chebyshev-accelerated Jacobi iteration for (1 - al2s lap) x = rhs:
//   y = x_{k-1} + gamma (rhs - A x_{k-1}) / diag,   x_k = x_{k-2} + omega_k (y - x_{k-2}),
// x_0 = x_{-1} = B^n (Bn), omega_1 = 1.  Iterate k lives in B when sweeps - k is even and in
// Bw otherwise, so the last one is B and x_{k-2} shares x_k's array (each cell reads its own
// old value before writing it).
__device__ __forceinline__ void relax_body(const FieldDesc& D, int i, int j, int kk, int k) {
    const FieldGeom& G = D.G;
    const int m = D.sweeps;
    double* out = ((m - k) % 2 == 0) ? D.B : D.Bw;
    const double* in = k == 1 ? D.Bn : (((m - k + 1) % 2 == 0) ? D.B : D.Bw);
    const double* prev = k <= 2 ? D.Bn : out;
    const double w = D.omega[k];
    const int q = lin(G, i, j, kk);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double* x = in + c * G.nc;
        const double xq = x[q];
        const double Ax = xq - D.al2s * lap(G, x, i, j, kk);
        const double y = xq + (D.R[c * G.nc + q] - Ax) * D.gdiag;
        const double p = prev[c * G.nc + q];
        out[c * G.nc + q] = p + w * (y - p);
    }
}

// E += c^2 dt (curl- (alpha B' + beta B) - mu0 J)
__device__ __forceinline__ void update_E_body(const FieldDesc& D, int i, int j, int k) {
    const FieldGeom& G = D.G;
    const int q = lin(G, i, j, k);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int d1 = (c + 1) % 3, d2 = (c + 2) % 3;
        double cn = ddn(G, D.B + d2 * G.nc, d1, i, j, k) - ddn(G, D.B + d1 * G.nc, d2, i, j, k);
        double co = ddn(G, D.Bn + d2 * G.nc, d1, i, j, k) - ddn(G, D.Bn + d1 * G.nc, d2, i, j, k);
        D.E[c * G.nc + q] += D.c2dt * (D.al * cn + D.be * co - D.mu0 * D.J[c * G.nc + q]);
    }
}

// Gauss-law filter pass, first half: r = div- E - (rho + rho_bg)/eps0 into R
__device__ __forceinline__ void gauss_res_body(const FieldDesc& D, int i, int j, int k) {
    const FieldGeom& G = D.G;
    const int q = lin(G, i, j, k);
    double dv = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) dv += ddn(G, D.E + c * G.nc, c, i, j, k);
    D.R[q] = dv - (D.rho[q] + D.rho_bg) * D.ieps0;
}

// second half: E_c += kappa d+_c r
__device__ __forceinline__ void gauss_corr_body(const FieldDesc& D, int i, int j, int k) {
    const FieldGeom& G = D.G;
    const int q = lin(G, i, j, k);
#pragma unroll
    for (int c = 0; c < 3; ++c) D.E[c * G.nc + q] += D.kappa * dup(G, D.R, c, i, j, k);
}

enum FieldPhase { PH_COPY = 0, PH_RHS = 1, PH_JACOBI = 2, PH_UPDATE_E = 3, PH_GAUSS_RES = 4, PH_GAUSS_CORR = 5 };

__device__ __forceinline__ void field_phase(const FieldDesc& D, int64_t b, int phase, int k) {
    int i, j, kk;
    if (!field_cell(D.G, b, threadIdx.x, i, j, kk)) return;
    if (phase == PH_COPY)
        copy_body(D, lin(D.G, i, j, kk));
    else if (phase == PH_RHS)
        rhs_body(D, i, j, kk);
    else if (phase == PH_JACOBI) {
        if (k <= D.sweeps) relax_body(D, i, j, kk, k);
    } else if (phase == PH_UPDATE_E)
        update_E_body(D, i, j, kk);
    else if (phase == PH_GAUSS_RES)
        gauss_res_body(D, i, j, kk);
    else
        gauss_corr_body(D, i, j, kk);
}

__global__ void __launch_bounds__(FIELD_BS) k_field(FieldDesc D, int phase, int k) {
    field_phase(D, blockIdx.x, phase, k);
}

// batched: block b belongs to run r with prefix[r] <= b < prefix[r+1] (prefix in blocks)
__global__ void __launch_bounds__(FIELD_BS) k_field_batch(const FieldDesc* __restrict__ T,
                                                          const int64_t* __restrict__ prefix, int nruns, int phase,
                                                          int k) {
    const int64_t b = blockIdx.x;
    const int r = find_segment(prefix, nruns, b);
    if (r < 0) return;
    field_phase(T[r], b - prefix[r], phase, k);
}

// Relaxation sweep, tiled (single-run path).  A block owns a 32 x 8 column of cells in x-y
// and marches over up to RX_ZC planes in z.  Each thread keeps the 2R+1 values of its own
// column around the current plane in registers (the z taps of the Laplacian) and the block
// stages the current plane of the tile plus an R-wide x-y ring in LDS (the x and y taps), so
// each value of the input comes from memory about once per plane instead of once per tap.
// The arithmetic and the order of the sums are those of relax_body, so both give the same
// bits (the batched path keeps relax_body).
constexpr int RX_TX = 32, RX_TY = 8, RX_ZC = 32;
constexpr int RX_BS = RX_TX * RX_TY;  // one thread per column of the tile
constexpr int64_t RX_MIN_BLOCKS = 1024 * 256 / RX_BS;  // 1024 threads' columns per CU

template <int R>
__global__ void __launch_bounds__(RX_BS) k_relax_tiled(FieldDesc D, int k) {
    constexpr int W = RX_TX + 2 * R, H = RX_TY + 2 * R;
    constexpr int NH = (W * H + RX_BS - 1) / RX_BS;  // ring entries a thread may stage per plane
    __shared__ double pl[W * H];
    const FieldGeom& G = D.G;
    const int n0 = G.n[0], n1 = G.n[1], n2 = G.n[2];
    const int nbx = (n0 + RX_TX - 1) / RX_TX, nby = (n1 + RX_TY - 1) / RX_TY;
    int b = blockIdx.x;
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby;
    const int bz = b / nby;
    const int i0 = bx * RX_TX, j0 = by * RX_TY, z0 = bz * RX_ZC;
    const int z1 = z0 + RX_ZC < n2 ? z0 + RX_ZC : n2;
    const int tx = threadIdx.x % RX_TX, ty = threadIdx.x / RX_TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool valid = i < n0 && j < n1;
    const int iw = nbw(i0, tx, n0, 1), jw = nbw(j0, ty, n1, 1);  // loads of idle threads wrap
    const int m = D.sweeps;
    double* out = ((m - k) % 2 == 0) ? D.B : D.Bw;
    const double* in = k == 1 ? D.Bn : (((m - k + 1) % 2 == 0) ? D.B : D.Bw);
    const double* prev = k <= 2 ? D.Bn : out;
    const double w = D.omega[k];
    const int nc = (int)G.nc;
    const int nxy = n0 * n1;
    // this thread's entries of the x-y ring around the tile: LDS index (-1: none) and
    // in-plane offset (periodic), the same for every plane
    int hl[NH], hg[NH];
#pragma unroll
    for (int e = 0; e < NH; ++e) {
        const int h = threadIdx.x + RX_BS * e;
        const int a = h % W, bb = h / W;
        const bool ring = h < W * H && !(a >= R && a < R + RX_TX && bb >= R && bb < R + RX_TY);
        hl[e] = ring ? h : -1;
        hg[e] = ring ? nbw(i0, a - R, n0, 1) + n0 * nbw(j0, bb - R, n1, 1) : 0;
    }
    const int own = valid ? lin(G, i, j, 0) : 0;
    for (int c = 0; c < 3; ++c) {
        const double* x = in + c * G.nc;
        const double* rhs = D.R + c * G.nc;
        const double* pv = prev + c * G.nc;
        // the loads of a plane are issued one plane ahead, so they are in flight while the
        // block works on the current one
        double q[2 * R + 1], hv[NH];
#pragma unroll
        for (int t = 0; t <= 2 * R; ++t) q[t] = x[lin(G, iw, jw, nbw(z0, t - R, n2, G.small))];
#pragma unroll
        for (int e = 0; e < NH; ++e) hv[e] = hl[e] >= 0 ? x[hg[e] + z0 * nxy] : 0.0;
        double rq = valid ? rhs[own + z0 * nxy] : 0.0;
        double pq = valid ? pv[own + z0 * nxy] : 0.0;
        for (int kz = z0; kz < z1; ++kz) {
            __syncthreads();  // the previous plane's LDS reads are done
            pl[(ty + R) * W + tx + R] = q[R];
#pragma unroll
            for (int e = 0; e < NH; ++e)
                if (hl[e] >= 0) pl[hl[e]] = hv[e];
            __syncthreads();
            const bool more = kz + 1 < z1;
            // the next plane's loads, unconditional (the last plane reloads its own plane, a lane
            // off the ring or the box reads the entries hg = 0 / own = 0) so that none waits at
            // a branch: they are first used by the next plane
            const int kn = more ? kz + 1 : kz;
            const double qn = x[lin(G, iw, jw, nbw(kn, R, n2, G.small))];
#pragma unroll
            for (int e = 0; e < NH; ++e) hv[e] = x[hg[e] + kn * nxy];
            const double rn = rhs[own + kn * nxy];
            const double pn = pv[own + kn * nxy];
            if (valid) {
                double sl = 0.0;
#pragma unroll
                for (int o = -R; o <= R; ++o) {
                    sl += G.L[0][o + R] * pl[(ty + R) * W + tx + R + o];
                    sl += G.L[1][o + R] * pl[(ty + R + o) * W + tx + R];
                    sl += G.L[2][o + R] * q[R + o];
                }
                const double xq = q[R];
                const double Ax = xq - D.al2s * sl;
                const double y = xq + (rq - Ax) * D.gdiag;
                out[c * nc + own + kz * nxy] = pq + w * (y - pq);
            }
            if (more) {
#pragma unroll
                for (int t = 0; t < 2 * R; ++t) q[t] = q[t + 1];
                q[2 * R] = qn;
                rq = rn;
                pq = pn;
            }
        }
        __syncthreads();
    }
}

// Right-hand side and E update, tiled the same way (single-run path): per component, each
// array the component's stencils read streams through the block one z plane at a time, its
// x-y ring staged in LDS when a stencil runs along x or y and a register window of z offsets
// kept when one runs along z; the next plane's loads are issued before the current plane is
// computed.  Sums are taken in the order of rhs_body and update_E_body (same bits).
struct TileCtx {
    int z0, z1, tx, ty, col, own, nxy, n2, small;
    bool valid;
};

template <int R>
struct Ring {  // this thread's entries of the x-y ring of a plane: LDS index (-1: none), offset
    static constexpr int W = RX_TX + 2 * R, H = RX_TY + 2 * R, NH = (W * H + RX_BS - 1) / RX_BS;
    int hl[NH], hg[NH];
};

template <int R>
__device__ __forceinline__ void tile_ctx(const FieldGeom& G, TileCtx& X, Ring<R>& g) {
    constexpr int W = Ring<R>::W, H = Ring<R>::H;
    const int n0 = G.n[0], n1 = G.n[1];
    const int nbx = (n0 + RX_TX - 1) / RX_TX, nby = (n1 + RX_TY - 1) / RX_TY;
    int b = blockIdx.x;
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby;
    const int bz = b / nby;
    const int i0 = bx * RX_TX, j0 = by * RX_TY;
    X.z0 = bz * RX_ZC;
    X.z1 = X.z0 + RX_ZC < G.n[2] ? X.z0 + RX_ZC : G.n[2];
    X.tx = threadIdx.x % RX_TX;
    X.ty = threadIdx.x / RX_TX;
    X.valid = i0 + X.tx < n0 && j0 + X.ty < n1;
    X.col = nbw(i0, X.tx, n0, 1) + n0 * nbw(j0, X.ty, n1, 1);  // idle threads load wrapped columns
    X.own = X.valid ? X.col : 0;
    X.nxy = n0 * n1;
    X.n2 = G.n[2];
    X.small = G.small;
#pragma unroll
    for (int e = 0; e < Ring<R>::NH; ++e) {
        const int h = threadIdx.x + RX_BS * e;
        const int a = h % W, bb = h / W;
        const bool ring = h < W * H && !(a >= R && a < R + RX_TX && bb >= R && bb < R + RX_TY);
        g.hl[e] = ring ? h : -1;
        g.hg[e] = ring ? nbw(i0, a - R, n0, 1) + n0 * nbw(j0, bb - R, n1, 1) : 0;
    }
}

// One array streamed through the planes: values at z offsets WLO..WHI of the thread's column
// around the current plane and, with PLANE, the current plane's ring for the LDS stage.
template <int R, int WLO, int WHI, bool PLANE>
struct ZStream {
    static constexpr int NW = WHI - WLO + 1, NH = Ring<R>::NH;
    const double* f;
    double w[NW];
    double hv[PLANE ? NH : 1];
    double wn;
    __device__ __forceinline__ void init(const double* src, const TileCtx& X, const Ring<R>& g) {
        f = src;
#pragma unroll
        for (int t = 0; t < NW; ++t) w[t] = f[X.col + X.nxy * nbw(X.z0, WLO + t, X.n2, X.small)];
        if constexpr (PLANE) {
#pragma unroll
            for (int e = 0; e < NH; ++e) hv[e] = g.hl[e] >= 0 ? f[g.hg[e] + X.z0 * X.nxy] : 0.0;
        }
    }
    __device__ __forceinline__ void stage(double* pl, const TileCtx& X, const Ring<R>& g) const {
        if constexpr (PLANE) {
            pl[(X.ty + R) * Ring<R>::W + X.tx + R] = w[-WLO];
#pragma unroll
            for (int e = 0; e < NH; ++e)
                if (g.hl[e] >= 0) pl[g.hl[e]] = hv[e];
        }
    }
    __device__ __forceinline__ void prefetch(int kz1, const TileCtx& X, const Ring<R>& g) {
        wn = f[X.col + X.nxy * nbw(kz1, WHI, X.n2, X.small)];
        if constexpr (PLANE) {
#pragma unroll
            for (int e = 0; e < NH; ++e)
                if (g.hl[e] >= 0) hv[e] = f[g.hg[e] + kz1 * X.nxy];
        }
    }
    __device__ __forceinline__ void shift() {
#pragma unroll
        for (int t = 0; t < NW - 1; ++t) w[t] = w[t + 1];
        w[NW - 1] = wn;
    }
    __device__ __forceinline__ double at(int o) const { return w[o - WLO]; }
};

// sum_m a_m (f[+m-1+UP] - f[-m+UP]) along axis AX (UP = 1: dup, UP = 0: ddn), from the staged
// plane (x, y) or the z window
template <int R, int M, int AX, int UP, class S>
__device__ __forceinline__ double dtile(const S& st, const double* pl, int c0, const double* a) {
    constexpr int step = AX == 0 ? 1 : Ring<R>::W;
    double s = 0.0;
#pragma unroll
    for (int m = 1; m <= M; ++m) {
        const int hi = m - 1 + UP, lo = -m + UP;
        if constexpr (AX == 2)
            s += a[m - 1] * (st.at(hi) - st.at(lo));
        else
            s += a[m - 1] * (pl[c0 + hi * step] - pl[c0 + lo * step]);
    }
    return s;
}

template <int M, int C>
__device__ __forceinline__ void rhs_tiled_comp(const FieldDesc& D, const TileCtx& X, const Ring<2 * M - 1>& g,
                                               double* lds) {
    constexpr int R = 2 * M - 1, WH = Ring<R>::W * Ring<R>::H;
    constexpr int d1 = (C + 1) % 3, d2 = (C + 2) % 3;
    constexpr bool uz = d1 == 2, vz = d2 == 2;  // which curl term differentiates along z
    const FieldGeom& G = D.G;
    ZStream<R, -R, R, true> sB;
    ZStream<R, uz ? -M + 1 : 0, uz ? M : 0, !uz> sEu, sJu;  // E_d2, J_d2 along d1
    ZStream<R, vz ? -M + 1 : 0, vz ? M : 0, !vz> sEv, sJv;  // E_d1, J_d1 along d2
    sB.init(D.Bn + C * G.nc, X, g);
    sEu.init(D.E + d2 * G.nc, X, g);
    sEv.init(D.E + d1 * G.nc, X, g);
    sJu.init(D.J + d2 * G.nc, X, g);
    sJv.init(D.J + d1 * G.nc, X, g);
    double *pB = lds, *pEu = lds + WH, *pEv = lds + 2 * WH, *pJu = lds + 3 * WH, *pJv = lds + 4 * WH;
    const int c0 = (X.ty + R) * Ring<R>::W + X.tx + R;
    for (int kz = X.z0; kz < X.z1; ++kz) {
        __syncthreads();  // the previous plane's LDS reads are done
        sB.stage(pB, X, g);
        sEu.stage(pEu, X, g);
        sEv.stage(pEv, X, g);
        sJu.stage(pJu, X, g);
        sJv.stage(pJv, X, g);
        __syncthreads();
        const bool more = kz + 1 < X.z1;
        if (more) {
            sB.prefetch(kz + 1, X, g);
            sEu.prefetch(kz + 1, X, g);
            sEv.prefetch(kz + 1, X, g);
            sJu.prefetch(kz + 1, X, g);
            sJv.prefetch(kz + 1, X, g);
        }
        if (X.valid) {
            double lp = 0.0;
#pragma unroll
            for (int o = -R; o <= R; ++o) {
                lp += G.L[0][o + R] * pB[c0 + o];
                lp += G.L[1][o + R] * pB[c0 + o * Ring<R>::W];
                lp += G.L[2][o + R] * sB.at(o);
            }
            double curlE = dtile<R, M, d1, 1>(sEu, pEu, c0, G.a[d1]) - dtile<R, M, d2, 1>(sEv, pEv, c0, G.a[d2]);
            double curlJ = dtile<R, M, d1, 1>(sJu, pJu, c0, G.a[d1]) - dtile<R, M, d2, 1>(sJv, pJv, c0, G.a[d2]);
            D.R[C * G.nc + X.own + (int64_t)kz * X.nxy] = sB.at(0) + D.cab * lp - D.dt * curlE + D.cj * curlJ;
        }
        if (more) {
            sB.shift();
            sEu.shift();
            sEv.shift();
            sJu.shift();
            sJv.shift();
        }
    }
}

template <int M, int C>
__device__ __forceinline__ void update_E_tiled_comp(const FieldDesc& D, const TileCtx& X, const Ring<2 * M - 1>& g,
                                                    double* lds) {
    constexpr int R = 2 * M - 1, WH = Ring<R>::W * Ring<R>::H;
    constexpr int d1 = (C + 1) % 3, d2 = (C + 2) % 3;
    constexpr bool uz = d1 == 2, vz = d2 == 2;
    const FieldGeom& G = D.G;
    ZStream<R, uz ? -M : 0, uz ? M - 1 : 0, !uz> sBu, sNu;  // B_d2, Bn_d2 along d1
    ZStream<R, vz ? -M : 0, vz ? M - 1 : 0, !vz> sBv, sNv;  // B_d1, Bn_d1 along d2
    ZStream<R, 0, 0, false> sE, sJ;
    sBu.init(D.B + d2 * G.nc, X, g);
    sBv.init(D.B + d1 * G.nc, X, g);
    sNu.init(D.Bn + d2 * G.nc, X, g);
    sNv.init(D.Bn + d1 * G.nc, X, g);
    sE.init(D.E + C * G.nc, X, g);
    sJ.init(D.J + C * G.nc, X, g);
    double *pBu = lds, *pBv = lds + WH, *pNu = lds + 2 * WH, *pNv = lds + 3 * WH;
    const int c0 = (X.ty + R) * Ring<R>::W + X.tx + R;
    for (int kz = X.z0; kz < X.z1; ++kz) {
        __syncthreads();
        sBu.stage(pBu, X, g);
        sBv.stage(pBv, X, g);
        sNu.stage(pNu, X, g);
        sNv.stage(pNv, X, g);
        __syncthreads();
        const bool more = kz + 1 < X.z1;
        if (more) {
            sBu.prefetch(kz + 1, X, g);
            sBv.prefetch(kz + 1, X, g);
            sNu.prefetch(kz + 1, X, g);
            sNv.prefetch(kz + 1, X, g);
            sE.prefetch(kz + 1, X, g);
            sJ.prefetch(kz + 1, X, g);
        }
        if (X.valid) {
            double cn = dtile<R, M, d1, 0>(sBu, pBu, c0, G.a[d1]) - dtile<R, M, d2, 0>(sBv, pBv, c0, G.a[d2]);
            double co = dtile<R, M, d1, 0>(sNu, pNu, c0, G.a[d1]) - dtile<R, M, d2, 0>(sNv, pNv, c0, G.a[d2]);
            D.E[C * G.nc + X.own + (int64_t)kz * X.nxy] =
                sE.at(0) + D.c2dt * (D.al * cn + D.be * co - D.mu0 * sJ.at(0));
        }
        if (more) {
            sBu.shift();
            sBv.shift();
            sNu.shift();
            sNv.shift();
            sE.shift();
            sJ.shift();
        }
    }
}

enum CurlKind { CK_RHS = 0, CK_UPDATE_E = 1 };

template <int M, int KIND>
__global__ void __launch_bounds__(RX_BS) k_curl_tiled(FieldDesc D) {
    constexpr int R = 2 * M - 1;
    __shared__ double lds[5 * Ring<R>::W * Ring<R>::H];
    TileCtx X;
    Ring<R> g;
    tile_ctx<R>(D.G, X, g);
    if constexpr (KIND == CK_RHS) {
        rhs_tiled_comp<M, 0>(D, X, g, lds);
        rhs_tiled_comp<M, 1>(D, X, g, lds);
        rhs_tiled_comp<M, 2>(D, X, g, lds);
    } else {
        update_E_tiled_comp<M, 0>(D, X, g, lds);
        update_E_tiled_comp<M, 1>(D, X, g, lds);
        update_E_tiled_comp<M, 2>(D, X, g, lds);
    }
}

template <int KIND>
static void launch_curl_tiled(const FieldDesc& D, int64_t blocks, hipStream_t st) {
    if (D.G.M == 3)
        hipLaunchKernelGGL((k_curl_tiled<3, KIND>), dim3((unsigned)blocks), dim3(RX_BS), 0, st, D);
    else if (D.G.M == 2)
        hipLaunchKernelGGL((k_curl_tiled<2, KIND>), dim3((unsigned)blocks), dim3(RX_BS), 0, st, D);
    else
        hipLaunchKernelGGL((k_curl_tiled<1, KIND>), dim3((unsigned)blocks), dim3(RX_BS), 0, st, D);
}

static int64_t relax_tiled_blocks(const FieldGeom& G) {
    return (int64_t)((G.n[0] + RX_TX - 1) / RX_TX) * ((G.n[1] + RX_TY - 1) / RX_TY) *
           ((G.n[2] + RX_ZC - 1) / RX_ZC);
}

static void fd_coeffs(int order, double a[3]) {
    a[0] = a[1] = a[2] = 0.0;
    if (order == 2) {
        a[0] = 1.0;
    } else if (order == 4) {
        a[0] = 9.0 / 8.0;
        a[1] = -1.0 / 24.0;
    } else {
        // 6th order; the normalisation a + 3b + 5c = 1 fixes a = 75/64
        a[0] = 75.0 / 64.0;
        a[1] = -25.0 / 384.0;
        a[2] = 3.0 / 640.0;
    }
}

static FieldGeom make_geom(const pp_run* r) {
    FieldGeom G{};
    for (int d = 0; d < 3; ++d) G.n[d] = r->p.n[d];
    G.nc = r->g.ncell;
    G.M = r->p.field_order / 2;
    double a[3];
    fd_coeffs(r->p.field_order, a);
    for (int d = 0; d < 3; ++d)
        for (int m = 0; m < 3; ++m) G.a[d][m] = a[m] / r->p.d[d];
    G.R = r->lap_r;
    for (int d = 0; d < 3; ++d)
        for (int o = 0; o < 2 * G.R + 1; ++o) G.L[d][o] = r->lap[d][o];
    const int nx = G.n[0];
    if (nx >= FIELD_BS) {
        G.xbits = 8;
        G.xchunks = (nx + FIELD_BS - 1) / FIELD_BS;
        G.rpb = 1;
    } else {
        G.xbits = 0;
        while ((1 << G.xbits) < nx) ++G.xbits;
        G.xchunks = 1;
        G.rpb = FIELD_BS >> G.xbits;
    }
    G.rows = G.n[1] * G.n[2];
    G.inv_ny = 1.0 / G.n[1];
    G.small = 0;
    for (int d = 0; d < 3; ++d)
        if (G.n[d] < G.R || G.n[d] < G.M) G.small = 1;
    return G;
}

static int64_t blocks_of(const FieldGeom& G) { return (int64_t)G.xchunks * ((G.rows + G.rpb - 1) / G.rpb); }

int64_t field_blocks(const pp_run* r) { return blocks_of(make_geom(r)); }

// Host set-up of the field-step constants: the composed Laplacian stencil (d- after d+,
// identical as a stencil to d+ after d-), the true diagonal of A = 1 - alpha^2 s lap on this
// periodic grid, and the relaxation.  A is circulant, so the Jacobi iteration matrix
// G = 1 - A / diag has its spectrum in [g0, g1] = [1 - amax/diag, 1 - 1/diag] exactly (amax
// the largest eigenvalue of A, from the stencil's symbol).  The relaxation is Jacobi
// extrapolated by gamma = 2 / (2 - g0 - g1), which centres that interval on 0 with radius
// r = (g1 - g0) / (2 - g0 - g1), and accelerated by Chebyshev semi-iteration (Golub and
// Varga 1961): after m sweeps the error is multiplied by at most 1 / T_m(1/r) (T_m the
// Chebyshev polynomial) and the residual by at most amax / T_m(1/r); m is the smallest
// count for which that is <= relax_tol.
static hipError_t relax_setup(pp_run* r, double dt, pp_run::RelaxSet& S);

hipError_t field_setup(pp_run* r) {
    double a[3];
    fd_coeffs(r->p.field_order, a);
    const int M = r->p.field_order / 2;
    const int R = 2 * M - 1;
    r->lap_r = R;
    for (int d = 0; d < 3; ++d) {
        for (int o = 0; o < 16; ++o) r->lap[d][o] = 0.0;
        const double id2 = 1.0 / (r->p.d[d] * r->p.d[d]);
        for (int m = 1; m <= M; ++m)
            for (int mp = 1; mp <= M; ++mp) {
                double cf = a[m - 1] * a[mp - 1] * id2;
                r->lap[d][(m + mp - 1) + R] += cf;
                r->lap[d][(m - mp) + R] -= cf;
                r->lap[d][(-m + mp) + R] -= cf;
                r->lap[d][(-m - mp + 1) + R] += cf;
            }
    }
    // Gauss-law filter damping: 1 / max over the grid's wave numbers of sum_d K_d^2, K_d the
    // symbol (2/d) sum_m a_m sin((m - 1/2) k) of the field-order first derivative
    double kmax2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        const int N = r->p.n[d];
        double best = 0.0;
        for (int mm = 0; mm < N; ++mm) {
            const double k = 2.0 * M_PI * mm / N;
            double sym = 0.0;
            for (int l = 1; l <= M; ++l) sym += a[l - 1] * sin((l - 0.5) * k);
            sym *= 2.0 / r->p.d[d];
            best = sym * sym > best ? sym * sym : best;
        }
        kmax2 += best;
    }
    r->gauss_kappa = kmax2 > 0.0 ? 1.0 / kmax2 : 0.0;
    // relaxation constants for each drift size the run steps with
    const double drifts[3] = {r->p.dt, FR_DRIFT[0] * r->p.dt, FR_DRIFT[2] * r->p.dt};
    for (int k = 0; k < r->nrs; ++k) {
        hipError_t e = relax_setup(r, drifts[k], r->rs[k]);
        if (e != hipSuccess) return e;
    }
    use_relax_set(r, 0);
    r->dt_kick = r->dt_drift = r->p.dt;
    return hipSuccess;
}

// Relaxation constants of one drift size dt (the operator depends on dt^2 only).
static hipError_t relax_setup(pp_run* r, double dt, pp_run::RelaxSet& S) {
    const int R = r->lap_r;
    const double s = r->p.c * r->p.c * dt * dt;
    const double al2s = r->p.alpha * r->p.alpha * s;
    double diag = 1.0, amax = 1.0;
    for (int d = 0; d < 3; ++d) {
        const int N = r->p.n[d];
        double fold0 = 0.0;
        for (int o = -R; o <= R; ++o)
            if (((o % N) + N) % N == 0) fold0 += r->lap[d][o + R];
        diag -= al2s * fold0;
        double mn = 0.0;
        for (int mm = 0; mm < N; ++mm) {
            double k = 2.0 * M_PI * mm / N, sym = 0.0;
            for (int o = -R; o <= R; ++o) sym += r->lap[d][o + R] * cos(o * k);
            if (sym < mn) mn = sym;
        }
        amax -= al2s * mn;
    }
    S.drift = dt;
    S.diagA = diag;
    const double g0 = 1.0 - amax / diag, g1 = 1.0 - 1.0 / diag;
    S.jac_rho = fmax(fabs(g0), fabs(g1));
    S.gamma = 2.0 / (2.0 - g0 - g1);
    const double rr = (g1 - g0) / (2.0 - g0 - g1);
    S.r = rr;
    // The paper relaxes until the residual is small (Sec. III.B).  After k sweeps the error is
    // reduced by at most 1/cosh(k acosh(1/r)) (Chebyshev); the residual rhs - A B_k = A e_k is
    // then reduced by at most that times the condition number of A, whose eigenvalues lie in
    // [1, amax] (1 - al2s lap with lap <= 0; the constant mode has eigenvalue 1).  The sweep
    // count is the smallest whose residual bound reaches relax_tol.
    const double kappa = amax;
    int sweeps = 1;
    double bound = 0.0;
    if (rr > 1e-300) {
        const double ac = acosh(1.0 / rr);
        for (sweeps = 1; sweeps < r->p.relax_max_iter; ++sweeps)
            if (kappa / cosh(sweeps * ac) <= r->p.relax_tol) break;
        bound = kappa / cosh(sweeps * ac);
    }
    S.sweeps = sweeps;
    S.bound = bound;
    S.converged = bound <= r->p.relax_tol;
    // omega_1 = 1, omega_2 = 1 / (1 - r^2/2), omega_{k+1} = 1 / (1 - r^2 omega_k / 4)
    const int n_om = r->p.relax_max_iter + 2;
    double* om = new (std::nothrow) double[n_om];
    if (!om) return hipErrorOutOfMemory;
    om[0] = 0.0;
    om[1] = 1.0;
    for (int k = 2; k < n_om; ++k) om[k] = k == 2 ? 1.0 / (1.0 - 0.5 * rr * rr) : 1.0 / (1.0 - 0.25 * rr * rr * om[k - 1]);
    hipError_t e = hipMemcpy(S.omega, om, n_om * sizeof(double), hipMemcpyHostToDevice);
    delete[] om;
    return e;
}

void use_relax_set(pp_run* r, int k) {
    const pp_run::RelaxSet& S = r->rs[k];
    r->diagA = S.diagA;
    r->jac_rho = S.jac_rho;
    r->relax_gamma = S.gamma;
    r->relax_r = S.r;
    r->jac_sweeps = S.sweeps;
    r->jac_bound = S.bound;
    r->jac_converged = S.converged;
    r->omega = S.omega;
    r->dt_drift = S.drift;
}

void field_desc(const pp_run* r, FieldDesc* D) {
    D->G = make_geom(r);
    const double c2 = r->p.c * r->p.c, dt = r->dt_drift, s = c2 * dt * dt;
    const double al = r->p.alpha, be = 1.0 - al;
    const double mu0 = 1.0 / (r->p.eps0 * c2);
    D->E = r->mesh.E;
    D->B = r->mesh.B;
    D->J = r->mesh.J;
    D->Bn = r->Bn;
    D->Bw = r->Bw;
    D->R = r->R;
    D->omega = r->omega;
    D->rho = r->rho;
    D->rho_bg = r->p.rho_background;
    D->ieps0 = 1.0 / r->p.eps0;
    D->kappa = r->gauss_kappa;
    D->cab = al * be * s;
    D->dt = dt;
    D->cj = al * c2 * mu0 * dt * dt;
    D->al2s = al * al * s;
    D->gdiag = r->relax_gamma / r->diagA;
    D->al = al;
    D->be = be;
    D->c2dt = c2 * dt;
    D->mu0 = mu0;
    D->sweeps = r->jac_sweeps;
}

size_t field_desc_size() { return sizeof(FieldDesc); }

hipError_t launch_field_step(pp_run* r) {
    FieldDesc D;
    field_desc(r, &D);
    const int bs = FIELD_BS;
    const dim3 grid((unsigned)blocks_of(D.G));
    // the tiled kernels need enough columns to fill the GPU; small boxes use the per-cell
    // ones (the same bits either way)
    const int64_t tb = relax_tiled_blocks(D.G);
    const dim3 rgrid((unsigned)tb);
    hipLaunchKernelGGL(k_field, grid, dim3(bs), 0, r->stream, D, (int)PH_COPY, 0);
    if (tb < RX_MIN_BLOCKS)
        hipLaunchKernelGGL(k_field, grid, dim3(bs), 0, r->stream, D, (int)PH_RHS, 0);
    else
        launch_curl_tiled<CK_RHS>(D, tb, r->stream);
    for (int k = 1; k <= D.sweeps; ++k) {
        if (tb < RX_MIN_BLOCKS)
            hipLaunchKernelGGL(k_field, grid, dim3(bs), 0, r->stream, D, (int)PH_JACOBI, k);
        else if (D.G.R == 5)
            hipLaunchKernelGGL(k_relax_tiled<5>, rgrid, dim3(RX_BS), 0, r->stream, D, k);
        else if (D.G.R == 3)
            hipLaunchKernelGGL(k_relax_tiled<3>, rgrid, dim3(RX_BS), 0, r->stream, D, k);
        else
            hipLaunchKernelGGL(k_relax_tiled<1>, rgrid, dim3(RX_BS), 0, r->stream, D, k);
    }
    if (tb < RX_MIN_BLOCKS)
        hipLaunchKernelGGL(k_field, grid, dim3(bs), 0, r->stream, D, (int)PH_UPDATE_E, 0);
    else
        launch_curl_tiled<CK_UPDATE_E>(D, tb, r->stream);
    note_relax_rhs(r);
    return hipGetLastError();
}

void note_relax_rhs(pp_run* r) {
    const double c2 = r->p.c * r->p.c, dt = r->dt_drift;
    r->rhs_valid = true;
    r->rhs_al2s = r->p.alpha * r->p.alpha * c2 * dt * dt;
}

// Residual of the relaxation actually reached (Sec. III.B: the paper relaxes to a residual):
// per cell and component r = R - (B - al2s lap B) with R the stored right-hand side, reduced
// to max |r| and max |R| (non-negative doubles compared as their bit patterns).
__device__ __forceinline__ void max_bits(double v, double* acc) {
    atomicMax((unsigned long long*)acc, (unsigned long long)__double_as_longlong(v));
}

__global__ void __launch_bounds__(FIELD_BS) k_relax_resid(FieldGeom G, const double* __restrict__ B,
                                                          const double* __restrict__ R, double al2s, double* acc) {
    __shared__ double red[2][FIELD_BS / 64];
    double rmax = 0.0, hmax = 0.0;
    int i, j, k;
    if (field_cell(G, blockIdx.x, threadIdx.x, i, j, k)) {
        const int q = lin(G, i, j, k);
        for (int c = 0; c < 3; ++c) {
            const double* x = B + c * G.nc;
            const double rhs = R[c * G.nc + q];
            const double Ax = x[q] - al2s * lap(G, x, i, j, k);
            rmax = fmax(rmax, fabs(rhs - Ax));
            hmax = fmax(hmax, fabs(rhs));
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        rmax = fmax(rmax, __shfl_xor(rmax, o));
        hmax = fmax(hmax, __shfl_xor(hmax, o));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = rmax;
        red[1][threadIdx.x >> 6] = hmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < FIELD_BS / 64; ++w) {
            rmax = fmax(rmax, red[0][w]);
            hmax = fmax(hmax, red[1][w]);
        }
        max_bits(rmax, acc);
        max_bits(hmax, acc + 1);
    }
}

hipError_t launch_relax_resid(pp_run* r, double* acc) {
    const FieldGeom G = make_geom(r);
    hipLaunchKernelGGL(k_relax_resid, dim3((unsigned)blocks_of(G)), dim3(FIELD_BS), 0, r->stream, G,
                       (const double*)r->mesh.B, (const double*)r->R, r->rhs_al2s, acc);
    return hipGetLastError();
}

// Gauss-law filter of a run (after its field step): rho of the current positions, then the
// passes, each a residual launch and a correction launch.
hipError_t launch_gauss_filter(pp_run* r) {
    r->rhs_valid = false;  // the passes keep their residual in R
    hipError_t e = deposit_rho_all(r);
    if (e != hipSuccess) return e;
    FieldDesc D;
    field_desc(r, &D);
    const dim3 grid((unsigned)blocks_of(D.G));
    for (int it = 0; it < r->p.gauss_filter_passes; ++it) {
        hipLaunchKernelGGL(k_field, grid, dim3(FIELD_BS), 0, r->stream, D, (int)PH_GAUSS_RES, 0);
        hipLaunchKernelGGL(k_field, grid, dim3(FIELD_BS), 0, r->stream, D, (int)PH_GAUSS_CORR, 0);
    }
    return hipGetLastError();
}

// Batched field step over n runs: table (device) of FieldDesc, prefix (device) of blocks.
hipError_t launch_field_step_batch(const void* table, const int64_t* prefix, int n, int64_t total_blocks,
                                   int max_sweeps, hipStream_t st) {
    if (n == 0 || total_blocks == 0) return hipSuccess;
    const FieldDesc* T = (const FieldDesc*)table;
    const dim3 grid((unsigned)total_blocks);
    hipLaunchKernelGGL(k_field_batch, grid, dim3(FIELD_BS), 0, st, T, prefix, n, (int)PH_COPY, 0);
    hipLaunchKernelGGL(k_field_batch, grid, dim3(FIELD_BS), 0, st, T, prefix, n, (int)PH_RHS, 0);
    for (int k = 1; k <= max_sweeps; ++k)
        hipLaunchKernelGGL(k_field_batch, grid, dim3(FIELD_BS), 0, st, T, prefix, n, (int)PH_JACOBI, k);
    hipLaunchKernelGGL(k_field_batch, grid, dim3(FIELD_BS), 0, st, T, prefix, n, (int)PH_UPDATE_E, 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// High-order current: on a periodic line the paper's construction (solve T dJ = dJ2 for the
// differences, prefix-sum, keep the line mean) equals J_O = T^{-1} J_2, because the
// high-order down derivative factors as T applied after the second-order one and T keeps
// line means (its symbol is 1 at k = 0).  T^{-1} is circulant with exponentially decaying
// coefficients; it is applied as a convolution along each component's own axis.
// ---------------------------------------------------------------------------------------
struct LineArgs {
    FieldGeom G;
    const double* coef[3];
    int len[3], off[3];
    // LDS form: W[c] lines of component c per block (a power of two, at most 64) and the
    // blocks of each component; W[0] == 0 selects the global-memory form
    int W[3];
    int64_t nb[3];
    const double* J2;
    double* J;
};

// Global-memory form (lines too long for the LDS copy): one thread per cell, the stencil
// read through the caches.
__device__ __forceinline__ void line_body(const LineArgs& A, int64_t b) {
    int ijk[3];
    if (!field_cell(A.G, b, threadIdx.x, ijk[0], ijk[1], ijk[2])) return;
    const int nc = (int)A.G.nc;
    const int q = lin(A.G, ijk[0], ijk[1], ijk[2]);
    const int stride[3] = {1, A.G.n[0], A.G.n[0] * A.G.n[1]};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double* src = A.J2 + (int64_t)c * nc;
        const int N = A.G.n[c];
        const int rowbase = q - ijk[c] * stride[c];
        double s = 0.0;
        int idx = ijk[c] + A.off[c];
        idx %= N;
        if (idx < 0) idx += N;
        for (int jj = 0; jj < A.len[c]; ++jj) {
            s += A.coef[c][jj] * src[rowbase + idx * stride[c]];
            if (++idx == N) idx = 0;
        }
        A.J[(int64_t)c * nc + q] = s;
    }
}

// LDS form.  A block takes W lines of one component along that component's axis, copies
// each line, extended by the stencil's wrap-around (ext = N + len - 1 values starting at
// offset off), into LDS with coalesced loads, then writes J[j] = sum_t coef[t] ext[j + t].
// x lines are rows (stored line by line, j fastest); y and z lines are taken W consecutive
// x at a time (stored with the W lines interleaved, x fastest), so loads and stores move
// whole rows or W-wide row segments.
constexpr int LINE_LDS_DOUBLES = 4608;  // 36 KiB: 16 lines of 256 cells plus the wrap-around
constexpr int LINE_BATCH = 8;           // loads per thread in flight while a block fills its lines

__device__ __forceinline__ void line_lds_body(const LineArgs& A, int64_t b, double* e) {
    const FieldGeom& G = A.G;
    int c = 0;
    if (b >= A.nb[0]) {
        b -= A.nb[0];
        c = 1;
        if (b >= A.nb[1]) {
            b -= A.nb[1];
            c = 2;
        }
    }
    if (c == 2 && b >= A.nb[2]) return;
    const int n0 = G.n[0], n1 = G.n[1];
    const int N = G.n[c], W = A.W[c], len = A.len[c], off = A.off[c];
    const int ext = N + len - 1;
    const int64_t nc = G.nc;
    const double* src = A.J2 + (int64_t)c * nc;
    double* dst = A.J + (int64_t)c * nc;
    // first line of the block and the line count / axis stride
    int64_t base0;
    int stride, nlines;
    if (c == 0) {
        const int64_t L0 = b * W;
        const int64_t rows = (int64_t)n1 * G.n[2];
        base0 = L0 * n0;
        stride = 1;
        nlines = (int)(rows - L0 < W ? rows - L0 : W);
    } else {
        const int nbx = (n0 + W - 1) / W;
        const int bx = (int)(b % nbx);
        const int64_t other = b / nbx;  // k for y lines, j for z lines
        const int i0 = bx * W;
        base0 = c == 1 ? i0 + (int64_t)n0 * n1 * other : i0 + (int64_t)n0 * other;
        stride = c == 1 ? n0 : n0 * n1;
        nlines = n0 - i0 < W ? n0 - i0 : W;
    }
    // line w starts at base0 + w * (x lines: n0, else 1)
    const int64_t lstep = c == 0 ? n0 : 1;
    const int total = ext * W;
    // global memory (not generic) loads, which the LDS stores need not wait behind
    const __attribute__((address_space(1))) double* gsrc = (const __attribute__((address_space(1))) double*)src;
    // LINE_BATCH loads per thread in flight before the first is stored; every lane loads (an
    // entry past the end or of a line past the last reads the block's first value and stores
    // nothing or zero), so that no load waits at a branch
    for (int q0 = threadIdx.x; q0 < total; q0 += LINE_BATCH * FIELD_BS) {
        double v[LINE_BATCH];
        int dst[LINE_BATCH];  // LDS entry, or -1 past the end
        bool live[LINE_BATCH];
#pragma unroll
        for (int t = 0; t < LINE_BATCH; ++t) {
            const int q = q0 + t * FIELD_BS;
            const int qc = q < total ? q : 0;
            int w, jj;
            if (c == 0) {
                w = qc / ext;
                jj = qc - w * ext;
            } else {
                jj = qc / W;
                w = qc - jj * W;
            }
            const int sidx = wrap_near(off + jj, N);
            live[t] = w < nlines;
            v[t] = gsrc[base0 + (live[t] ? w : 0) * lstep + (int64_t)sidx * stride];
            dst[t] = q < total ? q : -1;
        }
#pragma unroll
        for (int t = 0; t < LINE_BATCH; ++t)
            if (dst[t] >= 0) e[dst[t]] = live[t] ? v[t] : 0.0;
    }
    __syncthreads();
    const int outs = N * W;
    for (int q = threadIdx.x; q < outs; q += FIELD_BS) {
        int w, j, es, eb;
        if (c == 0) {
            w = q / N;
            j = q - w * N;
            eb = w * ext + j;
            es = 1;
        } else {
            j = q / W;
            w = q - j * W;
            eb = j * W + w;
            es = W;
        }
        if (w >= nlines) continue;
        // the coefficients are the same for the whole block: read-only, uniform (scalar) loads
        const __attribute__((address_space(4))) double* cf = (const __attribute__((address_space(4))) double*)A.coef[c];
        double s = 0.0;
        for (int t = 0; t < len; ++t) s += cf[t] * e[eb + t * es];
        dst[base0 + w * lstep + (int64_t)j * stride] = s;
    }
}

__device__ __forceinline__ void line_any(const LineArgs& A, int64_t b, double* e) {
    if (A.W[0] > 0)
        line_lds_body(A, b, e);
    else
        line_body(A, b);
}

__global__ void __launch_bounds__(FIELD_BS) k_line_solve(LineArgs A) {
    __shared__ double e[LINE_LDS_DOUBLES];
    line_any(A, blockIdx.x, e);
}

__global__ void __launch_bounds__(FIELD_BS) k_line_solve_batch(const LineArgs* __restrict__ T,
                                                               const int64_t* __restrict__ prefix, int nruns) {
    __shared__ double e[LINE_LDS_DOUBLES];
    const int64_t b = blockIdx.x;
    const int r = find_segment(prefix, nruns, b);
    if (r < 0) return;
    line_any(T[r], b - prefix[r], e);
}

// Host: coefficients of T^{-1} on a periodic line of N cells, by the discrete Fourier
// transform of 1 / T(k); truncated where they fall below 1e-18 of the centre value.
int line_setup_axis(int order, int N, double* coef_host, int* off) {
    double a[3];
    fd_coeffs(order, a);
    const int M = order / 2;
    double T[3] = {0, 0, 0};
    for (int l = 0; l < M; ++l)
        for (int m = l + 1; m <= M; ++m) T[l] += a[m - 1];
    // g(m) = 1/N sum_k cos(2 pi k m / N) / T(k)
    auto g = [&](int m) {
        double s = 0.0;
        for (int kk = 0; kk < N; ++kk) {
            double k = 2.0 * M_PI * kk / N;
            double sym = T[0];
            for (int l = 1; l < M; ++l) sym += 2.0 * T[l] * cos(l * k);
            s += cos(k * m) / sym;
        }
        return s / N;
    };
    // the coefficients decay geometrically down to the rounding noise of the sum (~1e-17);
    // keep them while two consecutive ones stand above 1e-16 of the centre value
    const double g0 = g(0);
    int Rr = 0;
    while (Rr < N / 2 && Rr < 63) {
        if (fabs(g(Rr + 1)) < 1e-16 * fabs(g0) && fabs(g(Rr + 2)) < 1e-16 * fabs(g0)) break;
        ++Rr;
    }
    if (2 * Rr + 1 >= N) {  // full circulant: offsets 0..N-1
        for (int m = 0; m < N; ++m) coef_host[m] = g(m);
        *off = 0;
        return N;
    }
    for (int m = -Rr; m <= Rr; ++m) coef_host[m + Rr] = g(m < 0 ? -m : m);
    *off = -Rr;
    return 2 * Rr + 1;
}

void line_desc(const pp_run* r, const double* J2, double* J, LineArgs* A) {
    A->G = make_geom(r);
    bool fits = true;
    for (int d = 0; d < 3; ++d) {
        A->coef[d] = r->line[d].coef;
        A->len[d] = r->line[d].len;
        A->off[d] = r->line[d].off;
        const int ext = r->p.n[d] + r->line[d].len - 1;
        int W = 64;
        while (W > 1 && (int64_t)W * ext > LINE_LDS_DOUBLES) W >>= 1;
        if ((int64_t)W * ext > LINE_LDS_DOUBLES) fits = false;
        A->W[d] = W;
        const int64_t n0 = r->p.n[0];
        if (d == 0)
            A->nb[d] = ((int64_t)r->p.n[1] * r->p.n[2] + W - 1) / W;
        else
            A->nb[d] = ((n0 + W - 1) / W) * (d == 1 ? r->p.n[2] : r->p.n[1]);
    }
    if (!fits) {
        A->W[0] = 0;
        A->nb[0] = blocks_of(A->G);
        A->nb[1] = A->nb[2] = 0;
    }
    A->J2 = J2;
    A->J = J;
}

size_t line_desc_size() { return sizeof(LineArgs); }

int64_t line_blocks(const pp_run* r) {
    LineArgs A;
    line_desc(r, nullptr, nullptr, &A);
    return A.nb[0] + A.nb[1] + A.nb[2];
}

hipError_t launch_line_solve(pp_run* r, const double* J2, double* J) {
    LineArgs A;
    line_desc(r, J2, J, &A);
    hipLaunchKernelGGL(k_line_solve, dim3((unsigned)(A.nb[0] + A.nb[1] + A.nb[2])), dim3(FIELD_BS), 0, r->stream,
                       A);
    return hipGetLastError();
}

hipError_t launch_line_solve_batch(const void* table, const int64_t* prefix, int n, int64_t total_blocks, hipStream_t st) {
    if (n == 0 || total_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_line_solve_batch, dim3((unsigned)total_blocks), dim3(FIELD_BS), 0, st, (const LineArgs*)table,
                       prefix, n);
    return hipGetLastError();
}

}  // namespace pp
