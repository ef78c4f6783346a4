// Plain FP64 form of steps 1-3 (Sec. III): one thread per particle, absolute FP64
// positions, fields read straight from global memory, current added with global FP64
// atomics.  It is the reference GPU form the tiled split-precision kernel is measured
// against.
#include "pp_device.hpp"
#include "pp_internal.hpp"

namespace pp {

struct Gpd64Args {
    int n[3];
    double d[3];      // cell size
    double dt, ic;    // drift time step (positions, current), 1/c
    double dtk;       // kick time step (momentum update)
    double h;         // q dt / m
    double krad;      // radiative cooling constant rad_tau q^2 / m (0: off)
    double fac[3];    // -q w d_c / dt, current prefactor per component
    int64_t np;
    double* pos[3];
    double* u[3];
    const double* E;
    const double* B;
    double* J;
    int64_t ncell;
    int32_t* flags;
    int pusher;
    int direct;       // PP_CURRENT_DIRECT: eq. "jj2" instead of the Esirkepov current
    double qw;        // q w (direct current)
};

template <int O>
__device__ __forceinline__ double gather1(const double* __restrict__ F, const int* ix, const int* iy, const int* iz,
                                          const double* wx, const double* wy, const double* wz, int nx, int nxy) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c <= O; ++c) {
        double accy = 0.0;
#pragma unroll
        for (int b = 0; b <= O; ++b) {
            const double* row = F + (int64_t)iz[c] * nxy + (int64_t)iy[b] * nx;
            double s = 0.0;
#pragma unroll
            for (int a = 0; a <= O; ++a) s += row[ix[a]] * wx[a];
            accy += s * wy[b];
        }
        acc += accy * wz[c];
    }
    return acc;
}

template <int O>
__global__ void __launch_bounds__(256) k_gpd64(Gpd64Args A) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.np) return;
    const int nx = A.n[0], ny = A.n[1], nz = A.n[2];
    const int nxy = nx * ny;
    const int64_t nc = A.ncell;

    double X0[3] = {A.pos[0][p], A.pos[1][p], A.pos[2][p]};
    V3<double> u{A.u[0][p], A.u[1][p], A.u[2][p]};

    // weights: centred (nodes at integers) and staggered (nodes at i + 1/2) per axis
    double wc[3][O + 1], ws[3][O + 1];
    int ic0[3][O + 1], is0[3][O + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int nd = A.n[d];
        int c0 = weights_abs<O>(X0[d], wc[d]);
        int s0 = weights_abs<O>(X0[d] - 0.5, ws[d]);
#pragma unroll
        for (int a = 0; a <= O; ++a) {
            ic0[d][a] = wrap(c0 + a, nd);
            is0[d][a] = wrap(s0 + a, nd);
        }
    }
    // eq. "pfields": E_x staggered along x, B_x staggered along y and z, cyclic
    V3<double> E, B;
    E.x = gather1<O>(A.E, is0[0], ic0[1], ic0[2], ws[0], wc[1], wc[2], nx, nxy);
    E.y = gather1<O>(A.E + nc, ic0[0], is0[1], ic0[2], wc[0], ws[1], wc[2], nx, nxy);
    E.z = gather1<O>(A.E + 2 * nc, ic0[0], ic0[1], is0[2], wc[0], wc[1], ws[2], nx, nxy);
    B.x = gather1<O>(A.B, ic0[0], is0[1], is0[2], wc[0], ws[1], ws[2], nx, nxy);
    B.y = gather1<O>(A.B + nc, is0[0], ic0[1], is0[2], ws[0], wc[1], ws[2], nx, nxy);
    B.z = gather1<O>(A.B + 2 * nc, is0[0], is0[1], ic0[2], ws[0], ws[1], wc[2], nx, nxy);

    const V3<double> um = u;
    if (A.pusher == PP_PUSH_BORIS)
        push_boris<double>(A.h, A.ic, E, B, u);
    else
        push_vay<double>(A.h, A.ic, E, B, u);
    if (A.krad != 0.0) rad_cool<double>(A.krad, A.dtk, A.ic, um, u);

    const double g = sqrt(1.0 + dot(u, u) * A.ic * A.ic);
    const double uu[3] = {u.x, u.y, u.z};
    double X1[3];
    int bad = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        X1[d] = X0[d] + A.dt * uu[d] / (g * A.d[d]);
        if (fabs(X1[d] - X0[d]) >= 1.0) bad |= PP_FLAG_CFL;
        if (!isfinite(X1[d]) || !isfinite(uu[d])) bad |= PP_FLAG_NONFINITE;
    }
    if (bad) {
        atomic_or_flag(A.flags, bad);
        return;
    }

    if (A.direct) {
        // direct current (eq. "jj2"): q w v_c W at J_c's staggered nodes, at the time-centred
        // position, with the gather's weights
        double Xm[3], wmc[3][O + 1], wms[3][O + 1];
        int imc[3][O + 1], ims[3][O + 1];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            Xm[d] = 0.5 * (X0[d] + X1[d]);
            const int c0 = weights_abs<O>(Xm[d], wmc[d]);
            const int s0 = weights_abs<O>(Xm[d] - 0.5, wms[d]);
#pragma unroll
            for (int a = 0; a <= O; ++a) {
                imc[d][a] = wrap(c0 + a, A.n[d]);
                ims[d][a] = wrap(s0 + a, A.n[d]);
            }
        }
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) {
            const double vq = A.qw * uu[comp] / g;
            double* Jc = A.J + comp * nc;
#pragma unroll
            for (int c = 0; c <= O; ++c) {
                const int k = comp == 2 ? ims[2][c] : imc[2][c];
                const double wz = comp == 2 ? wms[2][c] : wmc[2][c];
#pragma unroll
                for (int b = 0; b <= O; ++b) {
                    const int j = comp == 1 ? ims[1][b] : imc[1][b];
                    const double wzy = vq * wz * (comp == 1 ? wms[1][b] : wmc[1][b]);
#pragma unroll
                    for (int a = 0; a <= O; ++a) {
                        const int i = comp == 0 ? ims[0][a] : imc[0][a];
                        const double v = wzy * (comp == 0 ? wms[0][a] : wmc[0][a]);
                        if (v != 0.0) atomic_add_f64(Jc + (int64_t)i + (int64_t)nx * (j + (int64_t)ny * k), v);
                    }
                }
            }
        }
    } else {
    // Esirkepov current (Sec. III.C) on the common window of O+2 centred nodes per axis
    double S0[3][O + 2], DS[3][O + 2];
    int base[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double w0[O + 1], w1[O + 1];
        int a0 = weights_abs<O>(X0[d], w0);
        int a1 = weights_abs<O>(X1[d], w1);
        int b = a0 < a1 ? a0 : a1;
        base[d] = b;
        int o0 = a0 - b, o1 = a1 - b;  // 0 or 1
#pragma unroll
        for (int k = 0; k < O + 2; ++k) {
            int k0 = k - o0, k1 = k - o1;
            double s0 = (k0 >= 0 && k0 <= O) ? w0[k0 < 0 ? 0 : (k0 > O ? O : k0)] : 0.0;
            double s1 = (k1 >= 0 && k1 <= O) ? w1[k1 < 0 ? 0 : (k1 > O ? O : k1)] : 0.0;
            S0[d][k] = s0;
            DS[d][k] = s1 - s0;
        }
    }
    int idx[3][O + 2];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int k = 0; k < O + 2; ++k) idx[d][k] = wrap(base[d] + k, A.n[d]);

#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        const int d1 = comp == 0 ? 1 : (comp == 1 ? 2 : 0);
        const int d2 = comp == 0 ? 2 : (comp == 1 ? 0 : 1);
        double* Jc = A.J + comp * nc;
        const int strides[3] = {1, nx, nxy};
#pragma unroll
        for (int b = 0; b < O + 2; ++b) {
#pragma unroll
            for (int e = 0; e < O + 2; ++e) {
                double F = S0[d1][b] * S0[d2][e] + 0.5 * DS[d1][b] * S0[d2][e] + 0.5 * S0[d1][b] * DS[d2][e] +
                           DS[d1][b] * DS[d2][e] * (1.0 / 3.0);
                if (F == 0.0) continue;
                int64_t off = (int64_t)idx[d1][b] * strides[d1] + (int64_t)idx[d2][e] * strides[d2];
                double acc = 0.0;
#pragma unroll
                for (int a = 0; a <= O; ++a) {  // the last prefix (a = O+1) vanishes
                    acc += DS[comp][a] * F;
                    double v = A.fac[comp] * acc;
                    if (v != 0.0) atomic_add_f64(Jc + off + (int64_t)idx[comp][a] * strides[comp], v);
                }
            }
        }
    }
    }
    (void)ny;
    (void)nz;

#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double x = X1[d];
        const double nd = (double)A.n[d];
        if (x < 0.0) x += nd;
        if (x >= nd) x -= nd;
        A.pos[d][p] = x;
    }
    A.u[0][p] = u.x;
    A.u[1][p] = u.y;
    A.u[2][p] = u.z;
}

hipError_t launch_gpd64(pp_run* r, int s, double* J) {
    const Species& S = r->sp[s];
    if (S.n == 0) return hipSuccess;
    Gpd64Args A;
    for (int d = 0; d < 3; ++d) {
        A.n[d] = r->p.n[d];
        A.d[d] = r->p.d[d];
        A.pos[d] = (double*)S.cur.pos[d];
        A.u[d] = (double*)S.cur.u[d];
        A.fac[d] = -S.q * S.w * r->p.d[d] / r->dt_drift;
    }
    A.dt = r->dt_drift;
    A.dtk = r->dt_kick;
    A.ic = 1.0 / r->p.c;
    A.h = S.q * r->dt_kick / S.m;
    A.krad = r->p.rad_tau * S.q * S.q / S.m;
    A.np = S.n;
    A.E = r->mesh.E;
    A.B = r->mesh.B;
    A.J = J;
    A.ncell = r->g.ncell;
    A.flags = r->flags;
    A.pusher = r->p.pusher;
    A.direct = r->p.current_scheme == PP_CURRENT_DIRECT ? 1 : 0;
    A.qw = S.q * S.w;
    const int bs = 256;
    const int64_t nb = (S.n + bs - 1) / bs;
    if (r->p.shape_order == 2)
        hipLaunchKernelGGL(k_gpd64<2>, dim3((unsigned)nb), dim3(bs), 0, r->stream, A);
    else
        hipLaunchKernelGGL(k_gpd64<3>, dim3((unsigned)nb), dim3(bs), 0, r->stream, A);
    return hipGetLastError();
}

}  // namespace pp
