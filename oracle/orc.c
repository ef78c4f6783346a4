/*
 * orc.c -- plain FP64 CPU oracle for the particle step of the Photon-Plasma
 * relativistic particle-in-cell method (Haugboelle, Frederiksen & Nordlund,
 * "Photon-Plasma: a modern high-order particle-in-cell code", arXiv:1211.4575).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the HIP library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or helper with the GPU library.
 *
 * Everything is scalar FP64 in a fixed loop order.  Each function names the
 * passage of the paper it follows.  Conventions (the paper prints none of
 * these explicitly; they are the readings listed in the design notes):
 *   - positions X_d are in cell units, box [0, N_d), periodic;
 *   - Yee staggering (Sec. III, Fig. "yee"): rho at (i,j,k); E_x, J_x at
 *     (i+1/2,j,k); B_x at (i,j+1/2,k+1/2) and cyclic; a staggered array
 *     element [i] holds the value at i+1/2 in its staggered dimensions;
 *   - arrays are x-fastest: idx = i + nx*(j + ny*k); vector fields are three
 *     consecutive component blocks of ncell values.
 *   - units: mu0 = 1/(eps0 c^2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t n[3];         /* cells per dimension                              */
    double d[3];          /* cell size                                         */
    double dt, c, eps0;   /* time step, speed of light, vacuum permittivity    */
    int32_t shape_order;  /* B-spline weight order O: 0..3 (NGP, CIC, TSC, PCS)*/
    int32_t field_order;  /* finite-difference order: 2, 4 or 6                */
    double alpha;         /* implicit de-centering parameter                   */
    int32_t pusher;       /* 0 = Vay, 1 = Boris                                */
    double relax_tol;     /* relative residual target of the B relaxation      */
    int32_t relax_max_iter;
    double rho_background;/* fixed neutralising charge density                 */
    double rad_tau;       /* radiative cooling constant mu0 q^2 / (6 pi m c) for */
                          /* unit charge and mass (0: no cooling)                */
    int32_t current_scheme; /* 0 = charge-conserving (Esirkepov), 1 = direct     */
                          /* (eq. "jj2" at the time-centred position)            */
    int32_t gauss_passes; /* passes of the Gauss-law filter after the field step */
    int32_t time_order;   /* 2: leapfrog; 4: Forest-Ruth composition (whole-run  */
                          /* driver, orc.py); the kernels here take one substep */
    int32_t gauss_every;  /* filter after the field step of every k-th step only  */
                          /* (whole-run driver, orc.py; 0 or 1: every step)       */
} orc_params;

/* ------------------------------------------------------------------ */
/* indexing                                                             */
/* ------------------------------------------------------------------ */
static int wrapi(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

static size_t ncell(const orc_params* P) {
    return (size_t)P->n[0] * (size_t)P->n[1] * (size_t)P->n[2];
}

static size_t idx3(const orc_params* P, int i, int j, int k) {
    return (size_t)wrapi(i, P->n[0]) +
           (size_t)P->n[0] * ((size_t)wrapi(j, P->n[1]) + (size_t)P->n[1] * (size_t)wrapi(k, P->n[2]));
}

/* Stagger offsets (1/2 or 0) of each component, Sec. III (Yee lattice).   */
/* E and J: component d is shifted by 1/2 along d only.                   */
/* B: component d is shifted by 1/2 along the two other dimensions.       */
static double stagE(int comp, int dim) { return comp == dim ? 0.5 : 0.0; }
static double stagB(int comp, int dim) { return comp == dim ? 0.0 : 0.5; }

/* ------------------------------------------------------------------ */
/* B-spline weight functions W^O(delta), Sec. II, eqs. after            */
/* "weightfunction" (NGP, CIC, TSC, PCS); delta in cell units.          */
/* ------------------------------------------------------------------ */
double orc_W(int order, double delta) {
    double a = fabs(delta);
    switch (order) {
    case 0:
        return a <= 0.5 ? 1.0 : 0.0;
    case 1:
        return a < 1.0 ? 1.0 - a : 0.0;
    case 2:
        if (a < 0.5) return 0.75 - a * a;
        if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
        return 0.0;
    case 3:
        if (a < 1.0) return (4.0 - 6.0 * a * a + 3.0 * a * a * a) / 6.0;
        if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
        return 0.0;
    default:
        return 0.0;
    }
}

/* half-width of the weight's support, (O+1)/2 */
static double support_radius(int order) { return 0.5 * (order + 1); }

/* ------------------------------------------------------------------ */
/* Field at a particle, eq. "pfields": sum over mesh nodes of           */
/* F(node) W(node - X) in each dimension; a node of a component sits at */
/* i + stagger.  Every node whose weight can be non-zero is visited;    */
/* W itself returns zero outside the support.                           */
/* ------------------------------------------------------------------ */
static double gather_component(const orc_params* P, const double* F, const double s[3], const double X[3]) {
    const int O = P->shape_order;
    const double r = support_radius(O);
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = (int)floor(X[d] - s[d] - r);
        hi[d] = (int)ceil(X[d] - s[d] + r);
    }
    double sum = 0.0;
    for (int k = lo[2]; k <= hi[2]; ++k) {
        double wz = orc_W(O, k + s[2] - X[2]);
        if (wz == 0.0) continue;
        for (int j = lo[1]; j <= hi[1]; ++j) {
            double wy = orc_W(O, j + s[1] - X[1]);
            if (wy == 0.0) continue;
            for (int i = lo[0]; i <= hi[0]; ++i) {
                double wx = orc_W(O, i + s[0] - X[0]);
                if (wx == 0.0) continue;
                sum += F[idx3(P, i, j, k)] * wx * wy * wz;
            }
        }
    }
    return sum;
}

/* E and B at one particle position X (cell units). */
void orc_gather(const orc_params* P, const double* E, const double* B, const double X[3], double Ep[3], double Bp[3]) {
    const size_t nc = ncell(P);
    for (int comp = 0; comp < 3; ++comp) {
        double sE[3], sB[3];
        for (int d = 0; d < 3; ++d) {
            sE[d] = stagE(comp, d);
            sB[d] = stagB(comp, d);
        }
        Ep[comp] = gather_component(P, E + comp * nc, sE, X);
        Bp[comp] = gather_component(P, B + comp * nc, sB, X);
    }
}

/* ------------------------------------------------------------------ */
/* Momentum update, Sec. III.A.  The paper names the Vay pusher (its    */
/* default) and the Boris pusher and prints neither; these are the      */
/* published forms it cites (Vay 2008; Boris 1970).  u is the proper    */
/* velocity gamma*v; h = q dt / m.                                      */
/* ------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Vay: the velocity in v x B is the average of the old and new three-velocities;
 * the resulting quartic for the new Lorentz factor has a closed-form root. */
static void push_vay(double h, double c, const double E[3], const double B[3], double u[3]) {
    double g0 = sqrt(1.0 + dot3(u, u) / (c * c));
    double v[3] = {u[0] / g0, u[1] / g0, u[2] / g0};
    double vxB[3];
    cross3(v, B, vxB);
    double up[3];
    for (int d = 0; d < 3; ++d) up[d] = u[d] + h * (E[d] + 0.5 * vxB[d]);
    double tau[3] = {0.5 * h * B[0], 0.5 * h * B[1], 0.5 * h * B[2]};
    double tau2 = dot3(tau, tau);
    double ustar = dot3(up, tau) / c;
    double sigma = 1.0 + dot3(up, up) / (c * c) - tau2;
    double gn = sqrt(0.5 * (sigma + sqrt(sigma * sigma + 4.0 * (tau2 + ustar * ustar))));
    double t[3] = {tau[0] / gn, tau[1] / gn, tau[2] / gn};
    double s = 1.0 / (1.0 + dot3(t, t));
    double upt = dot3(up, t);
    double upxt[3];
    cross3(up, t, upxt);
    for (int d = 0; d < 3; ++d) u[d] = s * (up[d] + upt * t[d] + upxt[d]);
}

/* Boris: half electric kick, rotation about B using the proper-velocity
 * average, second half kick. */
static void push_boris(double h, double c, const double E[3], const double B[3], double u[3]) {
    double um[3];
    for (int d = 0; d < 3; ++d) um[d] = u[d] + 0.5 * h * E[d];
    double gm = sqrt(1.0 + dot3(um, um) / (c * c));
    double t[3] = {0.5 * h * B[0] / gm, 0.5 * h * B[1] / gm, 0.5 * h * B[2] / gm};
    double f = 2.0 / (1.0 + dot3(t, t));
    double s[3] = {f * t[0], f * t[1], f * t[2]};
    double umxt[3], uprime[3], upxs[3];
    cross3(um, t, umxt);
    for (int d = 0; d < 3; ++d) uprime[d] = um[d] + umxt[d];
    cross3(uprime, s, upxs);
    for (int d = 0; d < 3; ++d) u[d] = um[d] + upxs[d] + 0.5 * h * E[d];
}

void orc_push(int pusher, double q, double m, double dt, double c, const double E[3], const double B[3], double u[3]) {
    double h = q * dt / m;
    if (pusher == 1)
        push_boris(h, c, E, B, u);
    else
        push_vay(h, c, E, B, u);
}

/* Radiated power of a particle of proper velocity u and proper acceleration du/dt, over
 * mu0 q^2 / (6 pi c): the proper-velocity form of the Larmor-Lienard power (Sec. "Radiative
 * cooling", eq. "prad"): |du/dt|^2 + |du/dt x u|^2 / c^2. */
double orc_rad_bracket(double c, const double u[3], const double udot[3]) {
    double x[3];
    cross3(udot, u, x);
    return dot3(udot, udot) + dot3(x, x) / (c * c);
}

/* Radiative cooling of one step (Sec. "Radiative cooling", eqs. "prad", "udot" and the
 * explicit update that follows them): with u_m the proper velocity before the push and u the
 * one after the electromagnetic push, the time-centred state is u0 = (u + u_m)/2, gamma0 =
 * sqrt(1 + u0^2/c^2), the proper acceleration is (u - u_m)/dt, and
 *   u += -k (gamma0 / u0^2) [bracket] u0 dt,   k = rad_tau q^2 / m
 * (the cooling acts against u0; no iteration). */
void orc_rad_cool(double k, double dt, double c, const double u_m[3], double u[3]) {
    if (k == 0.0) return;
    double u0[3], ud[3];
    for (int d = 0; d < 3; ++d) {
        u0[d] = 0.5 * (u[d] + u_m[d]);
        ud[d] = (u[d] - u_m[d]) / dt;
    }
    const double u02 = dot3(u0, u0);
    if (!(u02 > 0.0)) return;
    const double g0 = sqrt(1.0 + u02 / (c * c));
    const double f = -k * g0 / u02 * orc_rad_bracket(c, u0, ud);
    for (int d = 0; d < 3; ++d) u[d] += f * u0[d] * dt;
}

/* Electromagnetic push followed by the cooling of one step (species charge q, mass m). */
void orc_push_rad(int pusher, double q, double m, double dt, double c, double rad_tau, const double E[3],
                  const double B[3], double u[3]) {
    double um[3] = {u[0], u[1], u[2]};
    orc_push(pusher, q, m, dt, c, E, B, u);
    orc_rad_cool(rad_tau * q * q / m, dt, c, um, u);
}

/* ------------------------------------------------------------------ */
/* Charge-conserving current of one particle moving X0 -> X1, Sec. III.C:*/
/* Esirkepov's directional split of the charge change (the paper cites  */
/* Esirkepov 2001 and prints no formula), then the per-particle prefix  */
/* sum valid for the second-order operator.  With S0, S1 the 1D weights */
/* at the old and new position and DS = S1 - S0:                        */
/*   W_x = DS_x (S0_y S0_z + DS_y S0_z / 2 + S0_y DS_z / 2 + DS_y DS_z/3)*/
/* and cyclic; J_x(i+1/2) = -(q w dx / dt) sum_{i' <= i} W_x(i').       */
/* Sign: chosen so that d_t rho + div J = 0 (eq. "cc1") holds.          */
/* J is accumulated (+=) into the three component blocks.               */
/* ------------------------------------------------------------------ */
#define ORC_MAXW 12
static void deposit_current_one(const orc_params* P, double q, double w, const double X0[3], const double X1[3], double* J) {
    const int O = P->shape_order;
    const double r = support_radius(O);
    const size_t nc = ncell(P);
    int lo[3], len[3];
    double S0[3][ORC_MAXW], DS[3][ORC_MAXW];
    for (int d = 0; d < 3; ++d) {
        double xmin = X0[d] < X1[d] ? X0[d] : X1[d];
        double xmax = X0[d] < X1[d] ? X1[d] : X0[d];
        lo[d] = (int)floor(xmin - r);
        int hi = (int)ceil(xmax + r);
        len[d] = hi - lo[d] + 1;
        for (int a = 0; a < len[d]; ++a) {
            double s0 = orc_W(O, lo[d] + a - X0[d]);
            double s1 = orc_W(O, lo[d] + a - X1[d]);
            S0[d][a] = s0;
            DS[d][a] = s1 - s0;
        }
    }
    for (int comp = 0; comp < 3; ++comp) {
        const int d1 = (comp + 1) % 3, d2 = (comp + 2) % 3;
        const double fac = -q * w * P->d[comp] / P->dt;
        double* Jc = J + comp * nc;
        for (int b = 0; b < len[d1]; ++b) {
            for (int e = 0; e < len[d2]; ++e) {
                double F = S0[d1][b] * S0[d2][e] + 0.5 * DS[d1][b] * S0[d2][e] + 0.5 * S0[d1][b] * DS[d2][e] +
                           DS[d1][b] * DS[d2][e] / 3.0;
                double acc = 0.0;
                for (int a = 0; a < len[comp]; ++a) {
                    acc += DS[comp][a] * F;
                    int ijk[3];
                    ijk[comp] = lo[comp] + a;
                    ijk[d1] = lo[d1] + b;
                    ijk[d2] = lo[d2] + e;
                    Jc[idx3(P, ijk[0], ijk[1], ijk[2])] += fac * acc;
                }
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Direct current of one particle (eq. "jj2"): J_d at its staggered      */
/* position (i+1/2 along d, integer along the other axes) receives      */
/* q w v_d W(node - X) with the same weights as the gather, taken at the */
/* time-centred position X = (X^n + X^{n+1})/2 and the three-velocity   */
/* v = u^{n+1/2} / gamma.  It does not satisfy eq. "cc1" in general.    */
/* ------------------------------------------------------------------ */
static void deposit_direct_one(const orc_params* P, double q, double w, const double X[3], const double v[3],
                               double* J) {
    const int O = P->shape_order;
    const double r = support_radius(O);
    const size_t nc = ncell(P);
    for (int comp = 0; comp < 3; ++comp) {
        double s[3] = {0.0, 0.0, 0.0};
        s[comp] = 0.5;
        int lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = (int)floor(X[d] - s[d] - r);
            hi[d] = (int)ceil(X[d] - s[d] + r);
        }
        for (int k = lo[2]; k <= hi[2]; ++k)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    double wt = orc_W(O, i + s[0] - X[0]) * orc_W(O, j + s[1] - X[1]) * orc_W(O, k + s[2] - X[2]);
                    if (wt != 0.0) J[comp * nc + idx3(P, i, j, k)] += q * w * v[comp] * wt;
                }
    }
}

/* Direct current of a single particle at X with three-velocity v (test hook). */
void orc_deposit_direct(const orc_params* P, double q, double w, const double X[3], const double v[3], double* J) {
    deposit_direct_one(P, q, w, X, v, J);
}

/* ------------------------------------------------------------------ */
/* Steps 1-3 of the time step (Sec. III list; eq. "pmotion" and the      */
/* position update of Sec. III.A) for one species:                      */
/*   gather E^n, B^n at X^n; push u^{n-1/2} -> u^{n+1/2};                */
/*   X^{n+1} = X^n + dt u^{n+1/2} / (gamma dx);                          */
/*   accumulate the second-order charge-conserving J (not zeroed here); */
/*   finally wrap X into [0, N).                                         */
/* pos and u are SoA: pos[d*n + p].  Returns a bit set: 1 = a particle   */
/* moved one cell or more along some axis, 2 = non-finite state.         */
/* ------------------------------------------------------------------ */
int orc_step_species_kd(const orc_params* P, double kick, double q, double m, double w, int64_t n, double* pos,
                        double* u, const double* E, const double* B, double* J);

int orc_step_species(const orc_params* P, double q, double m, double w, int64_t n, double* pos, double* u,
                     const double* E, const double* B, double* J) {
    return orc_step_species_kd(P, P->dt, q, m, w, n, pos, u, E, B, J);
}

/* One particle of the loop below: returns its flags; a non-finite particle is left as it
 * was and deposits nothing. */
static int step_one(const orc_params* P, double kick, double q, double m, double w, int64_t n, int64_t p, double* pos,
                    double* u, const double* E, const double* B, double* J) {
    int flags = 0;
    const double c = P->c;
    double X0[3], X1[3], up[3], Ep[3], Bp[3];
    for (int d = 0; d < 3; ++d) {
        X0[d] = pos[d * n + p];
        up[d] = u[d * n + p];
    }
    orc_gather(P, E, B, X0, Ep, Bp);
    orc_push_rad(P->pusher, q, m, kick, c, P->rad_tau, Ep, Bp, up);
    double g = sqrt(1.0 + dot3(up, up) / (c * c));
    for (int d = 0; d < 3; ++d) {
        X1[d] = X0[d] + P->dt * up[d] / (g * P->d[d]);
        if (fabs(X1[d] - X0[d]) >= 1.0) flags |= 1;
        if (!isfinite(X1[d]) || !isfinite(up[d])) flags |= 2;
    }
    if (flags & 2) return flags;
    if (P->current_scheme == 1) {
        double Xm[3], v[3];
        for (int d = 0; d < 3; ++d) {
            Xm[d] = 0.5 * (X0[d] + X1[d]);
            v[d] = up[d] / g;
        }
        deposit_direct_one(P, q, w, Xm, v, J);
    } else {
        deposit_current_one(P, q, w, X0, X1, J);
    }
    for (int d = 0; d < 3; ++d) {
        double x = fmod(X1[d], (double)P->n[d]);
        if (x < 0) x += P->n[d];
        if (x >= P->n[d]) x -= P->n[d];
        pos[d * n + p] = x;
        u[d * n + p] = up[d];
    }
    return flags;
}

/* The same with a momentum update (kick) over `kick` and the drift, current and position
 * update over P->dt: one substep of a composition scheme.
 * OpenMP mode (built with -fopenmp; the paper's shared-memory pattern, Sec. IX.B "OpenMP":
 * one current buffer per thread): the particles are split statically among the threads, each
 * thread deposits into its own zeroed copy of J, and the copies are added to J afterwards, for
 * every node in thread order.  Only the summation order of J differs from the plain build. */
int orc_step_species_kd(const orc_params* P, double kick, double q, double m, double w, int64_t n, double* pos,
                        double* u, const double* E, const double* B, double* J) {
    int flags = 0;
#ifdef _OPENMP
    const int nt = omp_get_max_threads();
    if (nt > 1) {
        const size_t n3 = 3 * ncell(P);
        double* priv = (double*)calloc((size_t)nt * n3, sizeof(double));
        if (priv) {
#pragma omp parallel reduction(| : flags)
            {
                double* Jt = priv + (size_t)omp_get_thread_num() * n3;
#pragma omp for schedule(static)
                for (int64_t p = 0; p < n; ++p) flags |= step_one(P, kick, q, m, w, n, p, pos, u, E, B, Jt);
            }
#pragma omp parallel for schedule(static)
            for (size_t i = 0; i < n3; ++i)
                for (int t = 0; t < nt; ++t) J[i] += priv[(size_t)t * n3 + i];
            free(priv);
            return flags;
        }
    }
#endif
    for (int64_t p = 0; p < n; ++p) flags |= step_one(P, kick, q, m, w, n, p, pos, u, E, B, J);
    return flags;
}

/* Current of a single particle moving X0 -> X1 (test hook). */
void orc_deposit_current(const orc_params* P, double q, double w, const double X0[3], const double X1[3], double* J) {
    deposit_current_one(P, q, w, X0, X1, J);
}

/* ------------------------------------------------------------------ */
/* Charge density, eq. "rho2": rho(node) += q w W(X - node), same       */
/* weights as the field gather.  Accumulates.                           */
/* ------------------------------------------------------------------ */
static void rho_one(const orc_params* P, double q, double w, int64_t n, int64_t p, const double* pos, double* rho) {
    const int O = P->shape_order;
    const double r = support_radius(O);
    double X[3];
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        X[d] = pos[d * n + p];
        lo[d] = (int)floor(X[d] - r);
        hi[d] = (int)ceil(X[d] + r);
    }
    for (int k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j)
            for (int i = lo[0]; i <= hi[0]; ++i) {
                double wt = orc_W(O, i - X[0]) * orc_W(O, j - X[1]) * orc_W(O, k - X[2]);
                if (wt != 0.0) rho[idx3(P, i, j, k)] += q * w * wt;
            }
}

/* OpenMP mode: one rho buffer per thread, added in thread order (as the current above). */
void orc_deposit_rho(const orc_params* P, double q, double w, int64_t n, const double* pos, double* rho) {
#ifdef _OPENMP
    const int nt = omp_get_max_threads();
    if (nt > 1) {
        const size_t nc = ncell(P);
        double* priv = (double*)calloc((size_t)nt * nc, sizeof(double));
        if (priv) {
#pragma omp parallel
            {
                double* rt = priv + (size_t)omp_get_thread_num() * nc;
#pragma omp for schedule(static)
                for (int64_t p = 0; p < n; ++p) rho_one(P, q, w, n, p, pos, rt);
            }
#pragma omp parallel for schedule(static)
            for (size_t i = 0; i < nc; ++i)
                for (int t = 0; t < nt; ++t) rho[i] += priv[(size_t)t * nc + i];
            free(priv);
            return;
        }
    }
#endif
    for (int64_t p = 0; p < n; ++p) rho_one(P, q, w, n, p, pos, rho);
}

/* ------------------------------------------------------------------ */
/* Staggered first derivatives, Sec. III.B ("ddyup" family).            */
/* Coefficients a_1..a_M (M = order/2):                                  */
/*   order 2: 1;  order 4: 9/8, -1/24;  order 6: 75/64, -25/384, 3/640.  */
/* The paper prints a = 25/21 for order 6; 75/64 is the value for which */
/* the operator is a first derivative (a + 3b + 5c = 1).  Order 4 is not */
/* printed; 9/8, -1/24 is the same Taylor family.                       */
/*  up:   out[i] (at i+1/2) = sum_m a_m (f[i+m]   - f[i-m+1]) / d        */
/*  down: out[i] (at i)     = sum_m a_m (g[i+m-1] - g[i-m])   / d        */
/* ------------------------------------------------------------------ */
static int fd_coeffs(int order, double a[3]) {
    a[0] = a[1] = a[2] = 0.0;
    if (order == 2) {
        a[0] = 1.0;
        return 1;
    }
    if (order == 4) {
        a[0] = 9.0 / 8.0;
        a[1] = -1.0 / 24.0;
        return 2;
    }
    a[0] = 75.0 / 64.0;
    a[1] = -25.0 / 384.0;
    a[2] = 3.0 / 640.0;
    return 3;
}

void orc_fd_coeffs(int order, double a[3]) { fd_coeffs(order, a); }

/* derivative along dim; up = 1 for the up-shifted operator. out must not alias f. */
static void deriv(const orc_params* P, const double* f, double* out, int dim, int up) {
    double a[3];
    const int M = fd_coeffs(P->field_order, a);
    const double inv = 1.0 / P->d[dim];
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < P->n[2]; ++k)
        for (int j = 0; j < P->n[1]; ++j)
            for (int i = 0; i < P->n[0]; ++i) {
                int ijk[3] = {i, j, k};
                double s = 0.0;
                for (int mm = 1; mm <= M; ++mm) {
                    int hiI[3] = {i, j, k}, loI[3] = {i, j, k};
                    if (up) {
                        hiI[dim] = ijk[dim] + mm;
                        loI[dim] = ijk[dim] - mm + 1;
                    } else {
                        hiI[dim] = ijk[dim] + mm - 1;
                        loI[dim] = ijk[dim] - mm;
                    }
                    s += a[mm - 1] * (f[idx3(P, hiI[0], hiI[1], hiI[2])] - f[idx3(P, loI[0], loI[1], loI[2])]);
                }
                out[idx3(P, i, j, k)] = s * inv;
            }
}

void orc_deriv(const orc_params* P, const double* f, double* out, int dim, int up) { deriv(P, f, out, dim, up); }

/* curl of a face-centred field (E or J) with up-shifted derivatives,
 * landing on the edges (B locations):  (curl+ F)_x = d+_y F_z - d+_z F_y */
void orc_curl_up(const orc_params* P, const double* F, double* out) {
    const size_t nc = ncell(P);
    double* t = (double*)malloc(nc * sizeof(double));
    for (int comp = 0; comp < 3; ++comp) {
        int d1 = (comp + 1) % 3, d2 = (comp + 2) % 3;
        deriv(P, F + d2 * nc, out + comp * nc, d1, 1);
        deriv(P, F + d1 * nc, t, d2, 1);
#pragma omp parallel for schedule(static)
        for (size_t q = 0; q < nc; ++q) out[comp * nc + q] -= t[q];
    }
    free(t);
}

/* curl of an edge field (B) with down-shifted derivatives, landing on faces */
void orc_curl_down(const orc_params* P, const double* F, double* out) {
    const size_t nc = ncell(P);
    double* t = (double*)malloc(nc * sizeof(double));
    for (int comp = 0; comp < 3; ++comp) {
        int d1 = (comp + 1) % 3, d2 = (comp + 2) % 3;
        deriv(P, F + d2 * nc, out + comp * nc, d1, 0);
        deriv(P, F + d1 * nc, t, d2, 0);
#pragma omp parallel for schedule(static)
        for (size_t q = 0; q < nc; ++q) out[comp * nc + q] -= t[q];
    }
    free(t);
}

/* divergence of a face-centred field, landing on cell centres (rho) */
void orc_div_down(const orc_params* P, const double* F, double* out) {
    const size_t nc = ncell(P);
    double* t = (double*)malloc(nc * sizeof(double));
    memset(out, 0, nc * sizeof(double));
    for (int d = 0; d < 3; ++d) {
        deriv(P, F + d * nc, t, d, 0);
#pragma omp parallel for schedule(static)
        for (size_t q = 0; q < nc; ++q) out[q] += t[q];
    }
    free(t);
}

/* ------------------------------------------------------------------ */
/* Gauss-law filter (Sec. "Charge conservation": the paper corrects E   */
/* iteratively after a non-conserving current and gives no formula).    */
/* Each pass: r = div- E - (rho + rho_bg)/eps0 at the cell centres, then */
/* E_d += kappa d+_d r.  A Fourier mode of r is multiplied by           */
/* 1 - kappa K(k)^2 (K^2 = sum_d K_d^2, K_d the symbol magnitude of the */
/* field-order first derivative), and kappa = 1 / max K^2 over the      */
/* grid's wave numbers removes the largest (Nyquist) error in one pass  */
/* and damps every other one.  The correction is a gradient: B and the  */
/* curl of E are untouched.                                             */
/* ------------------------------------------------------------------ */
double orc_gauss_kappa(const orc_params* P) {
    double a[3];
    const int M = fd_coeffs(P->field_order, a);
    double kmax2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        double best = 0.0;
        for (int m = 0; m < P->n[d]; ++m) {
            const double k = 2.0 * 3.14159265358979323846 * m / P->n[d];
            double sym = 0.0;
            for (int l = 1; l <= M; ++l) sym += a[l - 1] * sin((l - 0.5) * k);
            sym *= 2.0 / P->d[d];
            if (sym * sym > best) best = sym * sym;
        }
        kmax2 += best;
    }
    return kmax2 > 0.0 ? 1.0 / kmax2 : 0.0;
}

void orc_gauss_filter(const orc_params* P, double* E, const double* rho, int passes) {
    const size_t nc = ncell(P);
    const double kappa = orc_gauss_kappa(P);
    double* r = (double*)malloc(nc * sizeof(double));
    double* t = (double*)malloc(nc * sizeof(double));
    for (int it = 0; it < passes; ++it) {
        orc_div_down(P, E, r);
#pragma omp parallel for schedule(static)
        for (size_t q = 0; q < nc; ++q) r[q] -= (rho[q] + P->rho_background) / P->eps0;
        for (int d = 0; d < 3; ++d) {
            deriv(P, r, t, d, 1);
#pragma omp parallel for schedule(static)
            for (size_t q = 0; q < nc; ++q) E[d * nc + q] += kappa * t[q];
        }
    }
    free(r);
    free(t);
}

/* divergence of an edge field (B), landing on cell corners */
void orc_div_up(const orc_params* P, const double* F, double* out) {
    const size_t nc = ncell(P);
    double* t = (double*)malloc(nc * sizeof(double));
    memset(out, 0, nc * sizeof(double));
    for (int d = 0; d < 3; ++d) {
        deriv(P, F + d * nc, t, d, 1);
#pragma omp parallel for schedule(static)
        for (size_t q = 0; q < nc; ++q) out[q] += t[q];
    }
    free(t);
}

/* Laplacian of one component of an edge field (B): along a dimension where the
 * component sits on integer nodes, d- applied to d+; where it sits on half nodes,
 * d+ applied to d-.  This is the composition that makes curl+ curl- = grad div - lap
 * hold for the discrete operators (Sec. III.B). */
static void laplacian_B_component(const orc_params* P, int comp, const double* f, double* out) {
    const size_t nc = ncell(P);
    double* t1 = (double*)malloc(nc * sizeof(double));
    double* t2 = (double*)malloc(nc * sizeof(double));
    memset(out, 0, nc * sizeof(double));
    for (int d = 0; d < 3; ++d) {
        int half = stagB(comp, d) != 0.0;
        if (!half) {
            deriv(P, f, t1, d, 1);
            deriv(P, t1, t2, d, 0);
        } else {
            deriv(P, f, t1, d, 0);
            deriv(P, t1, t2, d, 1);
        }
#pragma omp parallel for schedule(static)
        for (size_t q = 0; q < nc; ++q) out[q] += t2[q];
    }
    free(t1);
    free(t2);
}

void orc_laplacian_B(const orc_params* P, const double* B, double* out) {
    const size_t nc = ncell(P);
    for (int comp = 0; comp < 3; ++comp) laplacian_B_component(P, comp, B + comp * nc, out + comp * nc);
}

/* ------------------------------------------------------------------ */
/* Field step, Sec. III.B, eqs. "bnplus1", "enplus1", "EllipticB".      */
/* With s = c^2 dt^2, beta = 1 - alpha, mu0 = 1/(eps0 c^2):             */
/*  (1 - alpha^2 s lap) B' = B + alpha beta s lap B - dt curl+ E        */
/*                           + alpha c^2 mu0 dt^2 curl+ J               */
/* (the J term enters with a plus sign: substituting "enplus1" into     */
/*  "bnplus1" gives +; the printed minus does not satisfy "bnplus1").   */
/* B' is found by relaxation (Jacobi) from the first guess B, stopping  */
/* when max|rhs - A B'| <= tol * max|rhs|.  Then                        */
/*  E' = E + c^2 dt (curl- (alpha B' + beta B) - mu0 J).                */
/* E, B updated in place.  Returns iterations; *resid = final relative  */
/* residual.                                                            */
/* ------------------------------------------------------------------ */
static void apply_A(const orc_params* P, const double* Bk, double* out, double* tmp) {
    const size_t n3 = 3 * ncell(P);
    const double s = P->c * P->c * P->dt * P->dt;
    orc_laplacian_B(P, Bk, tmp);
#pragma omp parallel for schedule(static)
    for (size_t q = 0; q < n3; ++q) out[q] = Bk[q] - P->alpha * P->alpha * s * tmp[q];
}

int orc_field_step(const orc_params* P, double* E, double* B, const double* J, double* resid_out) {
    const size_t nc = ncell(P), n3 = 3 * nc;
    const double c2 = P->c * P->c, s = c2 * P->dt * P->dt;
    const double al = P->alpha, be = 1.0 - P->alpha;
    const double mu0 = 1.0 / (P->eps0 * c2);
    double* rhs = (double*)calloc(n3, sizeof(double));
    double* tmp = (double*)calloc(n3, sizeof(double));
    double* tmp2 = (double*)calloc(n3, sizeof(double));
    double* Bn = (double*)calloc(n3, sizeof(double));
    double* Bk = (double*)calloc(n3, sizeof(double));
    double* AB = (double*)calloc(n3, sizeof(double));
    double diag[3];

    memcpy(Bn, B, n3 * sizeof(double));
    /* right-hand side */
    orc_laplacian_B(P, Bn, tmp);
#pragma omp parallel for schedule(static)
    for (size_t q = 0; q < n3; ++q) rhs[q] = Bn[q] + al * be * s * tmp[q];
    orc_curl_up(P, E, tmp);
#pragma omp parallel for schedule(static)
    for (size_t q = 0; q < n3; ++q) rhs[q] -= P->dt * tmp[q];
    orc_curl_up(P, J, tmp);
#pragma omp parallel for schedule(static)
    for (size_t q = 0; q < n3; ++q) rhs[q] += al * c2 * mu0 * P->dt * P->dt * tmp[q];

    /* diagonal of A on this periodic grid: (A e0)_0 for a unit impulse e0 */
    memset(Bk, 0, n3 * sizeof(double));
    for (int comp = 0; comp < 3; ++comp) Bk[comp * nc] = 1.0;
    apply_A(P, Bk, AB, tmp);
    for (int comp = 0; comp < 3; ++comp) diag[comp] = AB[comp * nc];

    double rhsmax = 0.0;
#pragma omp parallel for schedule(static) reduction(max : rhsmax)
    for (size_t q = 0; q < n3; ++q)
        if (fabs(rhs[q]) > rhsmax) rhsmax = fabs(rhs[q]);

    memcpy(Bk, Bn, n3 * sizeof(double)); /* first guess B^n */
    int it = 0;
    double res = 0.0;
    for (;;) {
        apply_A(P, Bk, AB, tmp);
        res = 0.0;
#pragma omp parallel for schedule(static) reduction(max : res)
        for (size_t q = 0; q < n3; ++q) {
            double rq = rhs[q] - AB[q];
            if (fabs(rq) > res) res = fabs(rq);
        }
        res = rhsmax > 0.0 ? res / rhsmax : res;
        if (res <= P->relax_tol || it >= P->relax_max_iter) break;
#pragma omp parallel for schedule(static)
        for (size_t g = 0; g < n3; ++g) Bk[g] += (rhs[g] - AB[g]) / diag[g / nc];
        ++it;
    }

    /* explicit E update */
#pragma omp parallel for schedule(static)
    for (size_t q = 0; q < n3; ++q) tmp2[q] = al * Bk[q] + be * Bn[q];
    orc_curl_down(P, tmp2, tmp);
#pragma omp parallel for schedule(static)
    for (size_t q = 0; q < n3; ++q) E[q] += c2 * P->dt * (tmp[q] - mu0 * J[q]);
    memcpy(B, Bk, n3 * sizeof(double));
    if (resid_out) *resid_out = res;
    free(rhs);
    free(tmp);
    free(tmp2);
    free(Bn);
    free(Bk);
    free(AB);
    return it;
}

/* ------------------------------------------------------------------ */
/* High-order charge-conserving current, Sec. III.C (eqs. "jj6d",        */
/* "penta"): per grid line along d, the second-order result J2 is       */
/* turned into its differences dJ2(i) = J2(i+1/2) - J2(i-1/2); the      */
/* banded system T dJ = dJ2 is solved on the line, with T the stencil   */
/* of the high-order down derivative in terms of differences            */
/*   order 6: [c, b+c, a+b+c, b+c, c];  order 4: [b, a+b, b];           */
/* then J(i+1/2) = prefix sum of dJ.  On a periodic line the system is  */
/* circulant and the prefix sum leaves the line mean undetermined; it   */
/* is fixed to the line mean of J2 (the paper's open-line construction  */
/* with a current-free virtual layer gives the same).  The solve is a   */
/* dense LU with partial pivoting of the circulant matrix.  Order 2:    */
/* identity.  J is overwritten.                                         */
/* ------------------------------------------------------------------ */
static void lu_factor(int n, double* A, int* piv) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > best) {
                best = fabs(A[i * n + k]);
                p = i;
            }
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; ++j) {
                double t = A[k * n + j];
                A[k * n + j] = A[p * n + j];
                A[p * n + j] = t;
            }
        for (int i = k + 1; i < n; ++i) {
            A[i * n + k] /= A[k * n + k];
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= A[i * n + k] * A[k * n + j];
        }
    }
}

static void lu_solve(int n, const double* A, const int* piv, double* b) {
    for (int k = 0; k < n; ++k) {
        int p = piv[k];
        if (p != k) {
            double t = b[k];
            b[k] = b[p];
            b[p] = t;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) b[i] -= A[i * n + j] * b[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) b[i] -= A[i * n + j] * b[j];
        b[i] /= A[i * n + i];
    }
}

void orc_current_high_order(const orc_params* P, double* J) {
    if (P->field_order == 2) return;
    double a[3];
    const int M = fd_coeffs(P->field_order, a);
    double T[3] = {0, 0, 0}; /* T[l] for |l| = 0..M-1: sum_{m > |l|} a_m */
    for (int l = 0; l < M; ++l)
        for (int mm = l + 1; mm <= M; ++mm) T[l] += a[mm - 1];
    const size_t nc = ncell(P);
    for (int dim = 0; dim < 3; ++dim) {
        const int N = P->n[dim];
        double* A = (double*)calloc((size_t)N * N, sizeof(double));
        int* piv = (int*)calloc(N, sizeof(int));
        for (int i = 0; i < N; ++i)
            for (int l = -(M - 1); l <= M - 1; ++l) A[i * N + wrapi(i + l, N)] += T[l < 0 ? -l : l];
        lu_factor(N, A, piv);
        double* Jc = J + dim * nc;
        int o1 = (dim + 1) % 3, o2 = (dim + 2) % 3;
        /* every line is independent (OpenMP mode: lines split among the threads) */
#pragma omp parallel
        {
            double* line = (double*)calloc(N, sizeof(double));
            double* dJ = (double*)calloc(N, sizeof(double));
#pragma omp for collapse(2) schedule(static)
            for (int e = 0; e < P->n[o2]; ++e)
                for (int b = 0; b < P->n[o1]; ++b) {
                    int ijk[3];
                    ijk[o1] = b;
                    ijk[o2] = e;
                    double mean2 = 0.0;
                    for (int i = 0; i < N; ++i) {
                        ijk[dim] = i;
                        line[i] = Jc[idx3(P, ijk[0], ijk[1], ijk[2])];
                        mean2 += line[i];
                    }
                    mean2 /= N;
                    for (int i = 0; i < N; ++i) dJ[i] = line[i] - line[wrapi(i - 1, N)];
                    lu_solve(N, A, piv, dJ);
                    double acc = 0.0, meanO = 0.0;
                    for (int i = 0; i < N; ++i) {
                        acc += dJ[i];
                        line[i] = acc;
                        meanO += acc;
                    }
                    meanO /= N;
                    for (int i = 0; i < N; ++i) {
                        ijk[dim] = i;
                        Jc[idx3(P, ijk[0], ijk[1], ijk[2])] = line[i] + (mean2 - meanO);
                    }
                }
            free(line);
            free(dJ);
        }
        free(A);
        free(piv);
    }
}

/* Threads the OpenMP build uses (1 for the plain build). */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Diagnostics (FP64).                                                  */
/* ------------------------------------------------------------------ */
/* kinetic energy sum_p w V m c^2 (gamma - 1) and momentum sum_p w V m u */
void orc_species_moments(const orc_params* P, double m, double w, int64_t n, const double* u, double* kin,
                         double mom[3]) {
    const double c = P->c, V = P->d[0] * P->d[1] * P->d[2];
    double K = 0.0, M[3] = {0, 0, 0};
    for (int64_t p = 0; p < n; ++p) {
        double up[3] = {u[p], u[n + p], u[2 * n + p]};
        double g = sqrt(1.0 + dot3(up, up) / (c * c));
        /* gamma - 1 = u^2 / (c^2 (gamma + 1)) avoids cancellation */
        K += w * V * m * dot3(up, up) / (g + 1.0);
        for (int d = 0; d < 3; ++d) M[d] += w * V * m * up[d];
    }
    *kin = K;
    for (int d = 0; d < 3; ++d) mom[d] = M[d];
}

/* field energies: sum eps0 |E|^2 V / 2 (also the x part) and sum |B|^2 V / (2 mu0) */
void orc_field_energy(const orc_params* P, const double* E, const double* B, double out[3]) {
    const size_t nc = ncell(P);
    const double V = P->d[0] * P->d[1] * P->d[2];
    const double mu0 = 1.0 / (P->eps0 * P->c * P->c);
    double UE = 0.0, UB = 0.0, UEx = 0.0;
    for (size_t q = 0; q < 3 * nc; ++q) {
        UE += 0.5 * P->eps0 * E[q] * E[q] * V;
        UB += 0.5 * B[q] * B[q] * V / mu0;
        if (q < nc) UEx += 0.5 * P->eps0 * E[q] * E[q] * V;
    }
    out[0] = UE;
    out[1] = UB;
    out[2] = UEx;
}
