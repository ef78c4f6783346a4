// Split-precision form of steps 1-3 (Sec. III), tiled.  Particles: int32 cell index +
// FP32 offset from the cell centre in [-1/2, 1/2) + FP32 proper velocity (the paper's
// integer cell + fraction storage, Sec. V.B), sorted by tile-major cell key.
//
// One workgroup (4 wavefronts) per tile of 64 cells:
//   1. stage E and B of the tile plus a 2-node halo from the FP64 mesh into LDS as FP32;
//   2. every lane owns one cell of the tile and walks that cell's particles; the four
//      wavefronts take every fourth particle of the cell.  A wavefront's 64 lanes therefore
//      work in 64 different cells, so the LDS atomics of one instruction never collide on
//      an address.  Per particle: gather (LDS) -> push (registers) -> move and
//      renormalise the split position -> Esirkepov current (registers) -> FP32 LDS
//      atomics into the tile's current block (3-node halo);
//   3. flush the current block to the FP64 mesh with global FP64 atomics (halo nodes
//      overlap neighbouring tiles), skipping untouched nodes.
// All species are processed by the same workgroup, so the fields are staged once.
#include "pp_device.hpp"
#include "pp_internal.hpp"

namespace pp {

struct Sp32 {
    const int32_t* off;  // bin starts
    int32_t* cell;
    float* pos[3];
    float* u[3];
    float h;       // q dt / m
    float fac[3];  // -q w d_c / dt
};

struct Gpd32Args {
    int n[3];
    int t[3];
    int nt[3];
    int64_t ntiles;
    int64_t nc;
    int fe[3];     // field LDS extents (1 on axes with a single cell)
    int ce[3];     // current LDS extents
    int flo[3];    // field halo below (0 on single-cell axes)
    int clo[3];    // current halo below
    float dt;
    float inv_d[3];
    float ic;
    int pusher;
    int nsp;
    Sp32 sp[PP_MAX_SPECIES];
    const double* E;
    const double* B;
    double* J;
    int32_t* flags;
    int per_xcd;   // tiles per XCD slot group
};

constexpr int GPD32_BS = 256;

// weights of the centred and staggered node sets for offset f in [-1/2, 1/2) of a
// particle in cell c; returned base offsets are relative to c.
template <int O>
__device__ __forceinline__ void split_weights(float f, float* wc, int& bc, float* ws, int& bs) {
    const float fl = floorf(f);  // -1 or 0
    if (O == 2) {
        weights_frac<2, float>(f, wc);  // nodes c-1..c+1
        bc = -1;
        weights_frac<2, float>(f - 0.5f - fl, ws);  // staggered nodes start at c-1+fl
        bs = -1 + (int)fl;
    } else {
        weights_frac<3, float>(f - fl, wc);  // nodes c-1+fl .. c+2+fl
        bc = -1 + (int)fl;
        weights_frac<3, float>(f + 0.5f, ws);  // staggered nodes c-2 .. c+1
        bs = -2;
    }
}

// centred weights of a position c + x, x in [-3/2, 3/2): first node offset and weights
template <int O>
__device__ __forceinline__ int centred_weights(float x, float* w) {
    if (O == 2) {
        float cn = floorf(x + 0.5f);
        weights_frac<2, float>(x - cn, w);
        return (int)cn - 1;
    } else {
        float f = floorf(x);
        weights_frac<3, float>(x - f, w);
        return (int)f - 1;
    }
}

template <int O>
__global__ void __launch_bounds__(GPD32_BS) k_gpd32(Gpd32Args A) {
    extern __shared__ float lds[];
    // XCD-aware tile order: consecutive workgroups go round-robin over the 8 XCDs, so give
    // each XCD a contiguous run of tiles (neighbouring tiles share halos in that XCD's L2).
    const int64_t b = blockIdx.x;
    const int64_t tile = (b & 7) * (int64_t)A.per_xcd + (b >> 3);
    if (tile >= A.ntiles) return;
    const int ti = (int)(tile % A.nt[0]);
    const int tj = (int)((tile / A.nt[0]) % A.nt[1]);
    const int tk = (int)(tile / ((int64_t)A.nt[0] * A.nt[1]));
    const int org[3] = {ti * A.t[0], tj * A.t[1], tk * A.t[2]};

    const int fsx = A.fe[0], fsy = A.fe[0] * A.fe[1];
    const int fvol = fsy * A.fe[2];
    const int csx = A.ce[0], csy = A.ce[0] * A.ce[1];
    const int cvol = csy * A.ce[2];
    float* fld = lds;               // 6 * fvol: Ex Ey Ez Bx By Bz
    float* cur = lds + 6 * fvol;    // 3 * cvol: Jx Jy Jz

    // 1. stage fields
    for (int q = threadIdx.x; q < 6 * fvol; q += GPD32_BS) {
        const int comp = q / fvol;
        const int r = q - comp * fvol;
        const int a = r % A.fe[0];
        const int bb = (r / A.fe[0]) % A.fe[1];
        const int c = r / fsy;
        const int gi = wrap(org[0] - A.flo[0] + a, A.n[0]);
        const int gj = wrap(org[1] - A.flo[1] + bb, A.n[1]);
        const int gk = wrap(org[2] - A.flo[2] + c, A.n[2]);
        const int64_t gq = (int64_t)gi + (int64_t)A.n[0] * (gj + (int64_t)A.n[1] * gk);
        const double* src = comp < 3 ? A.E + comp * A.nc : A.B + (comp - 3) * A.nc;
        fld[q] = (float)src[gq];
    }
    for (int q = threadIdx.x; q < 3 * cvol; q += GPD32_BS) cur[q] = 0.f;
    __syncthreads();

    // collapsed axes (a single cell) use stride 0 so every node offset maps to plane 0
    const int fst[3] = {A.n[0] > 1 ? 1 : 0, A.n[1] > 1 ? fsx : 0, A.n[2] > 1 ? fsy : 0};
    const int cst[3] = {A.n[0] > 1 ? 1 : 0, A.n[1] > 1 ? csx : 0, A.n[2] > 1 ? csy : 0};

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int lc[3] = {lane % A.t[0], (lane / A.t[0]) % A.t[1], lane / (A.t[0] * A.t[1])};
    const int64_t key0 = tile * TILE_CELLS;
    int bad_all = 0;

    for (int s = 0; s < A.nsp; ++s) {
        const Sp32& S = A.sp[s];
        const int32_t start = S.off[key0 + lane];
        const int32_t cnt = S.off[key0 + lane + 1] - start;
        for (int k = wv; k < cnt; k += 4) {
            const int32_t p = start + k;
            const int32_t cell = S.cell[p];
            float f[3] = {S.pos[0][p], S.pos[1][p], S.pos[2][p]};
            V3<float> u{S.u[0][p], S.u[1][p], S.u[2][p]};
            // decode and check the particle really lies in this tile's cell `lane`
            const int gi = cell % A.n[0];
            const int rr = cell / A.n[0];
            const int gj = rr % A.n[1];
            const int gk = rr / A.n[1];
            const int loc[3] = {gi - org[0], gj - org[1], gk - org[2]};
            if (loc[0] != lc[0] || loc[1] != lc[1] || loc[2] != lc[2] || !(f[0] >= -0.5f && f[0] < 0.5f) ||
                !(f[1] >= -0.5f && f[1] < 0.5f) || !(f[2] >= -0.5f && f[2] < 0.5f)) {
                bad_all |= PP_FLAG_OUT_OF_TILE;
                continue;
            }

            // gather (eq. "pfields") from the LDS field tile
            float wc[3][O + 1], ws[3][O + 1];
            int fc[3], fs[3];  // first LDS node index per axis (centred, staggered)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                int bc, bs;
                split_weights<O>(f[d], wc[d], bc, ws[d], bs);
                fc[d] = loc[d] + A.flo[d] + bc;
                fs[d] = loc[d] + A.flo[d] + bs;
            }
            V3<float> E, B;
            {
                auto G = [&](int comp, bool sx, bool sy, bool sz) {
                    const float* F = fld + comp * fvol;
                    const int bx = sx ? fs[0] : fc[0], by = sy ? fs[1] : fc[1], bz = sz ? fs[2] : fc[2];
                    const float* wx = sx ? ws[0] : wc[0];
                    const float* wy = sy ? ws[1] : wc[1];
                    const float* wz = sz ? ws[2] : wc[2];
                    // collapsed axes: nodes all at plane 0
                    float acc = 0.f;
#pragma unroll
                    for (int c = 0; c <= O; ++c) {
                        float accy = 0.f;
#pragma unroll
                        for (int b2 = 0; b2 <= O; ++b2) {
                            const float* row = F + (bz + c) * fst[2] + (by + b2) * fst[1] + bx * fst[0];
                            float sm = 0.f;
#pragma unroll
                            for (int a = 0; a <= O; ++a) sm += row[a * fst[0]] * wx[a];
                            accy += sm * wy[b2];
                        }
                        acc += accy * wz[c];
                    }
                    return acc;
                };
                E.x = G(0, true, false, false);
                E.y = G(1, false, true, false);
                E.z = G(2, false, false, true);
                B.x = G(3, false, true, true);
                B.y = G(4, true, false, true);
                B.z = G(5, true, true, false);
            }

            if (A.pusher == PP_PUSH_BORIS)
                push_boris<float>(S.h, A.ic, E, B, u);
            else
                push_vay<float>(S.h, A.ic, E, B, u);

            const float ig = rsqrtf(1.0f + dot(u, u) * A.ic * A.ic);
            const float uu[3] = {u.x, u.y, u.z};
            float x1[3];
            int bad = 0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const float dd = A.dt * uu[d] * ig * A.inv_d[d];
                if (!(fabsf(dd) < 1.0f)) bad |= isfinite(dd) ? PP_FLAG_CFL : PP_FLAG_NONFINITE;
                if (!isfinite(uu[d])) bad |= PP_FLAG_NONFINITE;
                x1[d] = f[d] + dd;  // new position relative to the old cell centre
            }
            if (bad) {
                bad_all |= bad;
                continue;
            }

            // Esirkepov current on the common window of O+2 centred nodes per axis
            float S0[3][O + 2], DS[3][O + 2];
            int wb[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                float w0[O + 1], w1[O + 1];
                const int a0 = centred_weights<O>(f[d], w0);
                const int a1 = centred_weights<O>(x1[d], w1);
                const int bmin = a0 < a1 ? a0 : a1;
                const int o0 = a0 - bmin, o1 = a1 - bmin;
#pragma unroll
                for (int kk = 0; kk < O + 2; ++kk) {
                    const int k0 = kk - o0, k1 = kk - o1;
                    const float s0 = (k0 >= 0 && k0 <= O) ? w0[k0 < 0 ? 0 : (k0 > O ? O : k0)] : 0.f;
                    const float s1 = (k1 >= 0 && k1 <= O) ? w1[k1 < 0 ? 0 : (k1 > O ? O : k1)] : 0.f;
                    S0[d][kk] = s0;
                    DS[d][kk] = s1 - s0;
                }
                wb[d] = loc[d] + A.clo[d] + bmin;  // first LDS current node
            }
#pragma unroll
            for (int comp = 0; comp < 3; ++comp) {
                const int d1 = comp == 0 ? 1 : (comp == 1 ? 2 : 0);
                const int d2 = comp == 0 ? 2 : (comp == 1 ? 0 : 1);
                float* Jc = cur + comp * cvol;
                const float fac = S.fac[comp];
#pragma unroll
                for (int bq = 0; bq < O + 2; ++bq) {
#pragma unroll
                    for (int e = 0; e < O + 2; ++e) {
                        const float Fq = S0[d1][bq] * S0[d2][e] + 0.5f * DS[d1][bq] * S0[d2][e] +
                                         0.5f * S0[d1][bq] * DS[d2][e] + DS[d1][bq] * DS[d2][e] * (1.0f / 3.0f);
                        const int rowo = (wb[d1] + bq) * cst[d1] + (wb[d2] + e) * cst[d2];
                        float acc = 0.f;
#pragma unroll
                        for (int a = 0; a <= O; ++a) {
                            acc += DS[comp][a] * Fq;
                            atomicAdd(Jc + rowo + (wb[comp] + a) * cst[comp], fac * acc);
                        }
                    }
                }
            }

            // renormalise: new cell = old cell + round(x1), offset back into [-1/2, 1/2)
            int nc3[3];
            float fn[3];
            const int gc[3] = {gi, gj, gk};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                float sh = floorf(x1[d] + 0.5f);
                float o = x1[d] - sh;
                // x1 + 1/2 can round up onto an integer: keep the offset in [-1/2, 1/2)
                if (o < -0.5f) {
                    o += 1.0f;
                    sh -= 1.0f;
                } else if (o >= 0.5f) {
                    o -= 1.0f;
                    sh += 1.0f;
                }
                fn[d] = o;
                int v = gc[d] + (int)sh;
                if (v < 0) v += A.n[d];
                if (v >= A.n[d]) v -= A.n[d];
                nc3[d] = v;
            }
            S.cell[p] = nc3[0] + A.n[0] * (nc3[1] + A.n[1] * nc3[2]);
            S.pos[0][p] = fn[0];
            S.pos[1][p] = fn[1];
            S.pos[2][p] = fn[2];
            S.u[0][p] = u.x;
            S.u[1][p] = u.y;
            S.u[2][p] = u.z;
        }
    }
    if (bad_all) atomic_or_flag(A.flags, bad_all);
    __syncthreads();

    // 3. flush the current block
    for (int q = threadIdx.x; q < 3 * cvol; q += GPD32_BS) {
        const float v = cur[q];
        if (v == 0.f) continue;
        const int comp = q / cvol;
        const int r = q - comp * cvol;
        const int a = r % A.ce[0];
        const int bb = (r / A.ce[0]) % A.ce[1];
        const int c = r / csy;
        const int gi = wrap(org[0] - A.clo[0] + a, A.n[0]);
        const int gj = wrap(org[1] - A.clo[1] + bb, A.n[1]);
        const int gk = wrap(org[2] - A.clo[2] + c, A.n[2]);
        atomic_add_f64(A.J + comp * A.nc + (int64_t)gi + (int64_t)A.n[0] * (gj + (int64_t)A.n[1] * gk), (double)v);
    }
}

size_t gpd32_lds_bytes(const pp_run* r) {
    int fv = 1, cv = 1;
    for (int d = 0; d < 3; ++d) {
        const bool single = r->p.n[d] == 1;
        fv *= single ? 1 : r->g.t[d] + FLD_LO + FLD_HI;
        cv *= single ? 1 : r->g.t[d] + CUR_LO + CUR_HI;
    }
    return (size_t)(6 * fv + 3 * cv) * sizeof(float);
}

hipError_t launch_gpd32(pp_run* r, double* J) {
    Gpd32Args A;
    for (int d = 0; d < 3; ++d) {
        A.n[d] = r->p.n[d];
        A.t[d] = r->g.t[d];
        A.nt[d] = r->g.nt[d];
        const bool single = r->p.n[d] == 1;
        A.fe[d] = single ? 1 : r->g.t[d] + FLD_LO + FLD_HI;
        A.ce[d] = single ? 1 : r->g.t[d] + CUR_LO + CUR_HI;
        A.flo[d] = single ? 0 : FLD_LO;
        A.clo[d] = single ? 0 : CUR_LO;
        A.inv_d[d] = (float)(1.0 / r->p.d[d]);
    }
    A.ntiles = r->g.ntiles;
    A.nc = r->g.ncell;
    A.dt = (float)r->p.dt;
    A.ic = (float)(1.0 / r->p.c);
    A.pusher = r->p.pusher;
    A.nsp = 0;
    for (int s = 0; s < PP_MAX_SPECIES; ++s) {
        const Species& S = r->sp[s];
        if (!S.active) continue;
        Sp32& D = A.sp[A.nsp++];
        D.off = S.offsets;
        D.cell = S.cur.cell;
        for (int d = 0; d < 3; ++d) {
            D.pos[d] = (float*)S.cur.pos[d];
            D.u[d] = (float*)S.cur.u[d];
            D.fac[d] = (float)(-S.q * S.w * r->p.d[d] / r->p.dt);
        }
        D.h = (float)(S.q * r->p.dt / S.m);
    }
    A.E = r->mesh.E;
    A.B = r->mesh.B;
    A.J = J;
    A.flags = r->flags;
    A.per_xcd = (int)((r->g.ntiles + 7) / 8);
    const size_t lds = gpd32_lds_bytes(r);
    const unsigned grid = (unsigned)(8 * (int64_t)A.per_xcd);
    if (r->p.shape_order == 2)
        hipLaunchKernelGGL(k_gpd32<2>, dim3(grid), dim3(GPD32_BS), lds, r->stream, A);
    else
        hipLaunchKernelGGL(k_gpd32<3>, dim3(grid), dim3(GPD32_BS), lds, r->stream, A);
    return hipGetLastError();
}

}  // namespace pp
