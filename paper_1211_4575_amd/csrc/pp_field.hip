// Field kernels: the implicit B / explicit E step (Sec. III.B, eqs. "bnplus1",
// "enplus1", "EllipticB") and the high-order current line solve (Sec. III.C, eqs.
// "jj6d", "penta").  Mesh arrays are FP64, x fastest, periodic.
#include "pp_device.hpp"
#include "pp_internal.hpp"

namespace pp {

struct FieldGeom {
    int n[3];
    int64_t nc;
    int M;           // half-width of the first-derivative stencil (order / 2)
    double a[3][3];  // a[axis][m-1] / d[axis]: first-derivative coefficients
    int R;           // Laplacian half-width 2M - 1
    double L[3][11]; // Laplacian stencil per axis, offsets -R..R
};

__device__ __forceinline__ int nb(int i, int o, int n) {
    int j = i + o;
    while (j < 0) j += n;
    while (j >= n) j -= n;
    return j;
}

__device__ __forceinline__ int64_t lin(const FieldGeom& G, int i, int j, int k) {
    return (int64_t)i + (int64_t)G.n[0] * ((int64_t)j + (int64_t)G.n[1] * k);
}

// up-shifted derivative along axis ax of f (values on integer nodes along ax) at cell (i,j,k):
// sum_m a_m (f[i+m] - f[i-m+1]) / d
__device__ __forceinline__ double dup(const FieldGeom& G, const double* __restrict__ f, int ax, int i, int j, int k) {
    int c[3] = {i, j, k};
    double s = 0.0;
    for (int m = 1; m <= G.M; ++m) {
        int hi[3] = {i, j, k}, lo[3] = {i, j, k};
        hi[ax] = nb(c[ax], m, G.n[ax]);
        lo[ax] = nb(c[ax], -m + 1, G.n[ax]);
        s += G.a[ax][m - 1] * (f[lin(G, hi[0], hi[1], hi[2])] - f[lin(G, lo[0], lo[1], lo[2])]);
    }
    return s;
}

// down-shifted derivative: sum_m a_m (g[i+m-1] - g[i-m]) / d
__device__ __forceinline__ double ddn(const FieldGeom& G, const double* __restrict__ f, int ax, int i, int j, int k) {
    int c[3] = {i, j, k};
    double s = 0.0;
    for (int m = 1; m <= G.M; ++m) {
        int hi[3] = {i, j, k}, lo[3] = {i, j, k};
        hi[ax] = nb(c[ax], m - 1, G.n[ax]);
        lo[ax] = nb(c[ax], -m, G.n[ax]);
        s += G.a[ax][m - 1] * (f[lin(G, hi[0], hi[1], hi[2])] - f[lin(G, lo[0], lo[1], lo[2])]);
    }
    return s;
}

__device__ __forceinline__ double lap(const FieldGeom& G, const double* __restrict__ f, int i, int j, int k) {
    double s = 0.0;
    for (int o = -G.R; o <= G.R; ++o) {
        s += G.L[0][o + G.R] * f[lin(G, nb(i, o, G.n[0]), j, k)];
        s += G.L[1][o + G.R] * f[lin(G, i, nb(j, o, G.n[1]), k)];
        s += G.L[2][o + G.R] * f[lin(G, i, j, nb(k, o, G.n[2]))];
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
    double cab, dt, cj;         // alpha beta s, dt, alpha c^2 mu0 dt^2   (s = c^2 dt^2)
    double al2s, inv_diag;      // alpha^2 s, 1 / diagonal
    double al, be, c2dt, mu0;   // alpha, beta, c^2 dt, mu0
    int sweeps;
};

__device__ __forceinline__ void cell_ijk(const FieldGeom& G, int64_t q, int& i, int& j, int& k) {
    i = (int)(q % G.n[0]);
    j = (int)((q / G.n[0]) % G.n[1]);
    k = (int)(q / ((int64_t)G.n[0] * G.n[1]));
}

__device__ __forceinline__ void copy_body(const FieldDesc& D, int64_t q) {
#pragma unroll
    for (int c = 0; c < 3; ++c) D.Bn[c * D.G.nc + q] = D.B[c * D.G.nc + q];
}

// rhs = B + alpha beta s lap B - dt curl+ E + alpha c^2 mu0 dt^2 curl+ J   (B = B^n from Bn)
__device__ __forceinline__ void rhs_body(const FieldDesc& D, int64_t q) {
    const FieldGeom& G = D.G;
    int i, j, k;
    cell_ijk(G, q, i, j, k);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int d1 = (c + 1) % 3, d2 = (c + 2) % 3;
        const double* Bc = D.Bn + c * G.nc;
        double curlE = dup(G, D.E + d2 * G.nc, d1, i, j, k) - dup(G, D.E + d1 * G.nc, d2, i, j, k);
        double curlJ = dup(G, D.J + d2 * G.nc, d1, i, j, k) - dup(G, D.J + d1 * G.nc, d2, i, j, k);
        D.R[c * G.nc + q] = Bc[q] + D.cab * lap(G, Bc, i, j, k) - D.dt * curlE + D.cj * curlJ;
    }
}

// sweep k (1-based) of Jacobi on (1 - al2s lap) x = rhs:  out = in + (rhs - in + al2s lap in) / diag.
// The sweeps alternate between B and Bw so that the last one writes B.
__device__ __forceinline__ void jacobi_body(const FieldDesc& D, int64_t q, int k) {
    const FieldGeom& G = D.G;
    const int m = D.sweeps;
    const double* in = k == 1 ? D.Bn : (((m - k + 1) % 2 == 0) ? D.B : D.Bw);
    double* out = ((m - k) % 2 == 0) ? D.B : D.Bw;
    int i, j, kk;
    cell_ijk(G, q, i, j, kk);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double* x = in + c * G.nc;
        double xq = x[q];
        double Ax = xq - D.al2s * lap(G, x, i, j, kk);
        out[c * G.nc + q] = xq + (D.R[c * G.nc + q] - Ax) * D.inv_diag;
    }
}

// E += c^2 dt (curl- (alpha B' + beta B) - mu0 J)
__device__ __forceinline__ void update_E_body(const FieldDesc& D, int64_t q) {
    const FieldGeom& G = D.G;
    int i, j, k;
    cell_ijk(G, q, i, j, k);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int d1 = (c + 1) % 3, d2 = (c + 2) % 3;
        double cn = ddn(G, D.B + d2 * G.nc, d1, i, j, k) - ddn(G, D.B + d1 * G.nc, d2, i, j, k);
        double co = ddn(G, D.Bn + d2 * G.nc, d1, i, j, k) - ddn(G, D.Bn + d1 * G.nc, d2, i, j, k);
        D.E[c * G.nc + q] += D.c2dt * (D.al * cn + D.be * co - D.mu0 * D.J[c * G.nc + q]);
    }
}

enum FieldPhase { PH_COPY = 0, PH_RHS = 1, PH_JACOBI = 2, PH_UPDATE_E = 3 };

__device__ __forceinline__ void field_phase(const FieldDesc& D, int64_t q, int phase, int k) {
    if (q >= D.G.nc) return;
    if (phase == PH_COPY)
        copy_body(D, q);
    else if (phase == PH_RHS)
        rhs_body(D, q);
    else if (phase == PH_JACOBI) {
        if (k <= D.sweeps) jacobi_body(D, q, k);
    } else
        update_E_body(D, q);
}

__global__ void __launch_bounds__(256) k_field(FieldDesc D, int phase, int k) {
    field_phase(D, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, phase, k);
}

// batched: block b belongs to run r with prefix[r] <= b < prefix[r+1] (prefix in blocks)
__global__ void __launch_bounds__(256) k_field_batch(const FieldDesc* __restrict__ T, const int64_t* __restrict__ prefix,
                                                     int nruns, int phase, int k) {
    const int64_t b = blockIdx.x;
    const int r = find_segment(prefix, nruns, b);
    if (r < 0) return;
    field_phase(T[r], (b - prefix[r]) * blockDim.x + threadIdx.x, phase, k);
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
    return G;
}

// Host set-up of the field-step constants: the composed Laplacian stencil (d- after d+,
// identical as a stencil to d+ after d-), the true diagonal of A = 1 - alpha^2 s lap on
// this periodic grid, and the number of Jacobi sweeps from the exact spectral radius of
// the (circulant) Jacobi iteration.
void field_setup(pp_run* r) {
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
    const double s = r->p.c * r->p.c * r->p.dt * r->p.dt;
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
    r->diagA = diag;
    double g1 = fabs(1.0 - 1.0 / diag), g2 = fabs(1.0 - amax / diag);
    double rho = g1 > g2 ? g1 : g2;
    r->jac_rho = rho;
    int sweeps = 1;
    if (rho > 0.0) {
        double want = log(r->p.relax_tol) / log(rho);
        sweeps = (int)ceil(want);
        if (sweeps < 1) sweeps = 1;
    }
    if (sweeps > r->p.relax_max_iter) sweeps = r->p.relax_max_iter;
    r->jac_sweeps = sweeps;
    r->jac_bound = rho > 0.0 ? pow(rho, sweeps) : 0.0;
}

void field_desc(const pp_run* r, FieldDesc* D) {
    D->G = make_geom(r);
    const double c2 = r->p.c * r->p.c, dt = r->p.dt, s = c2 * dt * dt;
    const double al = r->p.alpha, be = 1.0 - al;
    const double mu0 = 1.0 / (r->p.eps0 * c2);
    D->E = r->mesh.E;
    D->B = r->mesh.B;
    D->J = r->mesh.J;
    D->Bn = r->Bn;
    D->Bw = r->Bw;
    D->R = r->R;
    D->cab = al * be * s;
    D->dt = dt;
    D->cj = al * c2 * mu0 * dt * dt;
    D->al2s = al * al * s;
    D->inv_diag = 1.0 / r->diagA;
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
    const int bs = 256;
    const dim3 grid((unsigned)((D.G.nc + bs - 1) / bs));
    hipLaunchKernelGGL(k_field, grid, dim3(bs), 0, r->stream, D, (int)PH_COPY, 0);
    hipLaunchKernelGGL(k_field, grid, dim3(bs), 0, r->stream, D, (int)PH_RHS, 0);
    for (int k = 1; k <= D.sweeps; ++k) hipLaunchKernelGGL(k_field, grid, dim3(bs), 0, r->stream, D, (int)PH_JACOBI, k);
    hipLaunchKernelGGL(k_field, grid, dim3(bs), 0, r->stream, D, (int)PH_UPDATE_E, 0);
    return hipGetLastError();
}

// Batched field step over n runs: table (device) of FieldDesc, prefix (device) of blocks.
hipError_t launch_field_step_batch(const void* table, const int64_t* prefix, int n, int64_t total_blocks,
                                   int max_sweeps, hipStream_t st) {
    if (n == 0 || total_blocks == 0) return hipSuccess;
    const FieldDesc* T = (const FieldDesc*)table;
    const dim3 grid((unsigned)total_blocks);
    hipLaunchKernelGGL(k_field_batch, grid, dim3(256), 0, st, T, prefix, n, (int)PH_COPY, 0);
    hipLaunchKernelGGL(k_field_batch, grid, dim3(256), 0, st, T, prefix, n, (int)PH_RHS, 0);
    for (int k = 1; k <= max_sweeps; ++k)
        hipLaunchKernelGGL(k_field_batch, grid, dim3(256), 0, st, T, prefix, n, (int)PH_JACOBI, k);
    hipLaunchKernelGGL(k_field_batch, grid, dim3(256), 0, st, T, prefix, n, (int)PH_UPDATE_E, 0);
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
    int n[3];
    int64_t nc;
    const double* coef[3];
    int len[3], off[3];
    const double* J2;
    double* J;
};

__device__ __forceinline__ void line_body(const LineArgs& A, int64_t q) {
    if (q >= A.nc) return;
    const int ijk[3] = {(int)(q % A.n[0]), (int)((q / A.n[0]) % A.n[1]), (int)(q / ((int64_t)A.n[0] * A.n[1]))};
    const int64_t stride[3] = {1, A.n[0], (int64_t)A.n[0] * A.n[1]};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double* src = A.J2 + c * A.nc;
        const int N = A.n[c];
        const int64_t rowbase = q - (int64_t)ijk[c] * stride[c];
        double s = 0.0;
        int idx = nb(ijk[c], A.off[c], N);
        for (int jj = 0; jj < A.len[c]; ++jj) {
            s += A.coef[c][jj] * src[rowbase + (int64_t)idx * stride[c]];
            if (++idx == N) idx = 0;
        }
        A.J[c * A.nc + q] = s;
    }
}

__global__ void __launch_bounds__(256) k_line_solve(LineArgs A) {
    line_body(A, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void __launch_bounds__(256) k_line_solve_batch(const LineArgs* __restrict__ T, const int64_t* __restrict__ prefix,
                                                          int nruns) {
    const int64_t b = blockIdx.x;
    const int r = find_segment(prefix, nruns, b);
    if (r < 0) return;
    line_body(T[r], (b - prefix[r]) * blockDim.x + threadIdx.x);
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
    const double g0 = g(0);
    int Rr = 0;
    while (Rr < N / 2 && Rr < 63) {
        if (fabs(g(Rr + 1)) < 1e-18 * fabs(g0)) break;
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
    for (int d = 0; d < 3; ++d) {
        A->n[d] = r->p.n[d];
        A->coef[d] = r->line[d].coef;
        A->len[d] = r->line[d].len;
        A->off[d] = r->line[d].off;
    }
    A->nc = r->g.ncell;
    A->J2 = J2;
    A->J = J;
}

size_t line_desc_size() { return sizeof(LineArgs); }

hipError_t launch_line_solve(pp_run* r, const double* J2, double* J) {
    LineArgs A;
    line_desc(r, J2, J, &A);
    const int bs = 256;
    hipLaunchKernelGGL(k_line_solve, dim3((unsigned)((A.nc + bs - 1) / bs)), dim3(bs), 0, r->stream, A);
    return hipGetLastError();
}

hipError_t launch_line_solve_batch(const void* table, const int64_t* prefix, int n, int64_t total_blocks, hipStream_t st) {
    if (n == 0 || total_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_line_solve_batch, dim3((unsigned)total_blocks), dim3(256), 0, st, (const LineArgs*)table, prefix, n);
    return hipGetLastError();
}

}  // namespace pp
