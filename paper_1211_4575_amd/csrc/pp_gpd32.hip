// Split-precision form of steps 1-3 (Sec. III), tiled.  Particles: int32 cell index +
// FP32 offset inside the cell + FP32 proper velocity (the paper's integer cell + fraction
// storage, Sec. V.B).  The offset is measured from the nearest node (lo = -1/2) for quadratic
// weights and from the node below (lo = 0) for cubic weights and lies in [lo, lo + 1), so
// that the centred support starts one node below the cell; a particle whose last
// displacement, repeated (scaled by the ratio of the next drift to this one inside a
// composed step), would take it across the lower face of its cell is kept in the cell
// below with its offset in [lo + 1, lo + 2).  Then the current window of the next step
// (old and new support) starts 2 nodes below the cell for almost every particle.
// Particles are stored per tile in pairs of ranks, 64 pairs to a chunk of 128 slots (see
// pp_sort.hip): the 64 first and the 64 second particles of a chunk each sit in different
// cells of the tile, in a full round all 64 cells in order, so the 64 lanes of a wavefront
// touch 64 aligned stencils, which the padded LDS layout spreads over all banks.
//
// One workgroup (4 wavefronts) per tile of 64 cells:
//   1. stage E and B of the tile plus a 2-node halo from the FP64 mesh into LDS as FP32;
//   2. each wavefront takes 64 consecutive particles at a time (coalesced loads and
//      stores): gather (LDS) -> push (registers) -> move and renormalise the split
//      position -> Esirkepov current (registers) -> LDS accumulation of the tile's current
//      block (halo of 2 nodes below and O + 1 above);
//   3. flush the current block to the global accumulator with 64-bit integer atomics.
// For the next sort each particle also gets its rank among the particles of its new cell:
// an LDS counter per destination cell of the tile's neighbourhood hands out ranks inside
// the tile, one global atomic per destination cell then reserves the tile's range in that
// cell's count, and a second pass over the tile's particles adds the range start.
// Current accumulation is exact 64-bit fixed point.  Each contribution P_a * F * fac is
// formed in FP64 by one fused multiply-add with the rounding constant 1.5*2^52, whose bit
// pattern is then (constant bits + round(contribution * 2^e)); that pattern is added to the
// LDS block with an integer atomic (integer LDS atomics run at full rate on gfx950, FP32 LDS
// atomics at a small fraction of it).  The constant's share of a node's sum only touches bit
// 51 and above, so the sum of the rounded contributions is the sign-extended low 51 bits,
// recovered when the block is flushed; the scale 2^e (from the largest particle count of any
// tile) keeps every node's sum below 2^50 in magnitude.  The global accumulator adds the
// recovered integers, so the current is the exact sum of the rounded contributions,
// independent of summation order (bitwise deterministic).  All species are processed by the
// same workgroup.
#include "pp_device.hpp"
#include "pp_internal.hpp"

namespace pp {

struct Sp32 {
    const int32_t* start;  // tile starts (ntiles + 1)
    int32_t* cnt;          // particles per cell of the new positions (for the next sort)
    int32_t* rank;         // rank of each particle in its new cell (for the next sort)
    // A sort leaves the new order as a permutation: slot q of the tile order holds the
    // particle at index perm[q] of the input arrays, and the kernel writes slot q of the
    // output arrays (it moves the particles as it updates them).  perm == nullptr: in place.
    const int32_t* perm;
    const int32_t* cell;
    const float* pos[3];
    const float* u[3];
    int32_t* cell_o;
    float* pos_o[3];
    float* u_o[3];
    const int64_t* id;  // tags moved with the permutation (nullptr: none or in place)
    int64_t* id_o;
    float h;        // q dt / m
    float krad;     // radiative cooling constant rad_tau q^2 / m (0: off)
    double fac[3];  // -q w d_c / dt
    double qw;      // q w (direct current)
};

struct Gpd32Args {
    int n[3];
    int t[3];
    int nt[3];
    int64_t ntiles;
    int64_t nc;
    int fe[3], ce[3];  // LDS extents (runtime-shape kernel)
    int flo[3], clo[3];
    float dt;   // drift: positions and current
    float dtk;  // kick: momentum update (radiative cooling included)
    float pred; // next drift / this drift: the next displacement expected from this one
    float inv_d[3];
    float ic;
    int pusher;
    int nsp;
    Sp32 sp[PP_MAX_SPECIES];
    const double* E;
    const double* B;
    unsigned long long* Jq;  // fixed-point current accumulator (3 * nc)
    const double* qscale;    // 2^e (device, set by k_fixed_scale)
    int32_t* flags;
    int per_xcd;
    int sext[3];  // destination-cell window per axis (tile + 2 below + 2 above; 1 if collapsed)
    int nslots;   // sext[0] * sext[1] * sext[2]
    int direct;   // PP_CURRENT_DIRECT: eq. "jj2" instead of the Esirkepov current
};

constexpr int GPD32_BS = 256;
constexpr int STAGE_BATCH = 8;  // field loads / current reads a thread issues before the first wait
constexpr double ROUND_MAGIC = 6755399441055744.0;  // 1.5 * 2^52
constexpr unsigned long long LOW51 = (1ull << 51) - 1ull;
constexpr long long BIT50 = 1ll << 50;

// sum of rounded contributions held in the low 51 bits of an accumulated bit pattern
__device__ __forceinline__ long long fixed_sum(unsigned long long v) {
    return (long long)((v & LOW51) ^ (unsigned long long)BIT50) - BIT50;
}

// Padded row and plane strides (64-bit elements) of the current block.  The 64 lanes of a
// round hold one particle per cell, so an accumulation instruction touches 64 addresses laid
// out like the tile's cells.  A 64-bit LDS access covers a pair of the 32 banks and is served
// 16 lanes at a time; lanes 16g..16g+15 are the 4x4 cells of one z layer (or two x rows of
// a flat 8x8 tile), and a row stride of 12 (24) puts those 16 addresses on 16 different bank
// pairs.  A plane stride that is a multiple of 16 keeps a window moved by one z layer on its
// bank pairs.
constexpr int cur_row_444 = 12;
constexpr int cur_plane_444(int O) { return O == 2 ? 112 : 128; }
constexpr int cur_row_881 = 24;
// Row and plane strides (floats) of the field tile of a 4x4x4 tile (cubic weights: padded
// from 9 and 81, which measured a few per cent faster).
constexpr int fld_row_444(int O) { return O == 3 ? 10 : O + 6; }
constexpr int fld_plane_444(int O) { return O == 3 ? 90 : (O + 6) * (O + 6); }

// LDS layout of a tile: compile-time for the common shapes, runtime otherwise.  A
// single-cell axis is collapsed (extent 1, stride 0): every node offset maps to plane 0.
// The current block is indexed x + crow*y + cplane*z (padding entries stay zero).
template <int O, int TX, int TY, int TZ, bool CZ>
struct TileCT {
    static constexpr int tx = TX, ty = TY, tz = TZ;
    static constexpr int flox = FLD_LO, floy = FLD_LO, floz = CZ ? 0 : FLD_LO;
    static constexpr int clox = cur_lo(O), cloy = cur_lo(O), cloz = CZ ? 0 : cur_lo(O);
    static constexpr int fex = TX + FLD_LO + fld_hi(O), fey = TY + FLD_LO + fld_hi(O);
    static constexpr int fez = CZ ? 1 : TZ + FLD_LO + fld_hi(O);
    static constexpr int cex = TX + cur_lo(O) + cur_hi(O), cey = TY + cur_lo(O) + cur_hi(O);
    static constexpr int cez = CZ ? 1 : TZ + cur_lo(O) + cur_hi(O);
    static constexpr bool f444 = TX == 4 && TY == 4 && TZ == 4 && !CZ;
    static constexpr int frow = f444 ? fld_row_444(O) : fex;
    static constexpr int fplane = f444 ? fld_plane_444(O) : frow * fey;
    static constexpr int fsx = 1, fsy = frow, fsz = CZ ? 0 : fplane;
    static constexpr bool t444 = TX == 4 && TY == 4 && TZ == 4 && !CZ;
    static constexpr bool t881 = TX == 8 && TY == 8 && CZ;
    static constexpr int crow = t444 ? cur_row_444 : (t881 ? cur_row_881 : cex);
    static constexpr int cplane = t444 ? cur_plane_444(O) : crow * cey;
    static_assert(crow >= cex, "current row padding");
    static_assert(cplane >= crow * cey, "current plane padding");
    static constexpr int csx = 1, csy = crow, csz = CZ ? 0 : cplane;
    static_assert(frow >= fex && fplane >= frow * fey, "field tile padding");
    static constexpr int fvol = fplane * fez, cvol = cplane * cez;
    // two particles per lane (the paired deposit) on cubic tiles; flat tiles keep one per
    // lane, whose smaller register set leaves room for more resident wavefronts
    static constexpr bool pairs = t444;
    static constexpr bool flat = CZ;  // one field plane: the gather's z taps read the same nodes
    __device__ TileCT(const Gpd32Args&) {}
};

struct TileRT {
    static constexpr bool pairs = false;
    static constexpr bool flat = false;
    int tx, ty, tz;
    int flox, floy, floz, clox, cloy, cloz;
    int fex, fey, fez, cex, cey, cez;
    int fsx, fsy, fsz, csx, csy, csz;
    int crow, cplane, frow, fplane;
    int fvol, cvol;
    __device__ TileRT(const Gpd32Args& A) {
        tx = A.t[0];
        ty = A.t[1];
        tz = A.t[2];
        flox = A.flo[0];
        floy = A.flo[1];
        floz = A.flo[2];
        clox = A.clo[0];
        cloy = A.clo[1];
        cloz = A.clo[2];
        fex = A.fe[0];
        fey = A.fe[1];
        fez = A.fe[2];
        cex = A.ce[0];
        cey = A.ce[1];
        cez = A.ce[2];
        fsx = A.n[0] > 1 ? 1 : 0;
        frow = fex;
        fplane = fex * fey;
        fsy = A.n[1] > 1 ? frow : 0;
        fsz = A.n[2] > 1 ? fplane : 0;
        crow = cex;
        cplane = cex * cey;
        csx = A.n[0] > 1 ? 1 : 0;
        csy = A.n[1] > 1 ? crow : 0;
        csz = A.n[2] > 1 ? cplane : 0;
        fvol = fplane * fez;
        cvol = cplane * cez;
    }
};

// Lower end of the offset range of the split form (see the header).
template <int O>
__device__ __forceinline__ constexpr float off_lo() {
    return O == 2 ? -0.5f : 0.0f;
}

template <int O>
__device__ __forceinline__ bool offset_ok(float f) {
    return f >= off_lo<O>() && f < off_lo<O>() + 2.0f;
}

// weights of the centred and staggered node sets for offset f of a particle in cell c;
// returned base offsets are relative to c.
template <int O>
__device__ __forceinline__ void split_weights(float f, float* wc, int& bc, float* ws, int& bs) {
    if (O == 2) {
        const float cn = floorf(f + 0.5f);  // nearest node: 0 or 1
        weights_frac<2, float>(f - cn, wc);  // nodes c-1+cn .. c+1+cn
        bc = -1 + (int)cn;
        const float cs = floorf(f);  // nearest staggered node c+cs+1/2, cs in -1..1
        weights_frac<2, float>(f - 0.5f - cs, ws);
        bs = -1 + (int)cs;
    } else {
        const float fl = floorf(f);  // 0 or 1
        weights_frac<3, float>(f - fl, wc);  // nodes c-1+fl .. c+2+fl
        bc = -1 + (int)fl;
        const float y = f - 0.5f;  // position on the staggered lattice
        const float fy = floorf(y);  // -1, 0 or 1
        weights_frac<3, float>(y - fy, ws);
        bs = -1 + (int)fy;
    }
}

// centred weights of a position c + x, x in (-3/2, 3/2): first node offset and weights
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

typedef __attribute__((address_space(3))) const float lds_cfloat;

template <int O, class TL>
__device__ __forceinline__ float gather_comp(const float* __restrict__ F, const TL& L, int bx, int by, int bz,
                                             const float* wx, const float* wy, const float* wz) {
    lds_cfloat* base = (lds_cfloat*)(F + bz * L.fsz + by * L.fsy + bx * L.fsx);
    float acc = 0.f;
#pragma unroll
    for (int c = 0; c <= O; ++c) {
        // one address per plane, kept opaque: the plane's nodes are then small immediate
        // offsets of it (LDS paired reads reach 255 words; the stencil spans more than that).
        // A flat tile has one plane, whose reads the compiler shares between the z taps.
        lds_cfloat* plane = base + c * L.fsz;
        if constexpr (!TL::flat) asm volatile("" : "+v"(plane));
        float accy = 0.f;
#pragma unroll
        for (int b = 0; b <= O; ++b) {
            float s = 0.f;
#pragma unroll
            for (int a = 0; a <= O; ++a) s += plane[b * L.fsy + a * L.fsx] * wx[a];
            accy += s * wy[b];
        }
        acc += accy * wz[c];
    }
    return acc;
}

// Rank of a particle among those bound for its destination cell: rel = destination cell
// relative to the tile origin (unwrapped), gcell = its linear index.  Inside the tile's
// window the rank comes from the LDS counter of that cell (slot << 20 | rank in the tile;
// completed after the tile by the cell's range start); otherwise from the global count
// directly (bit 31 set).
__device__ __forceinline__ int32_t dest_rank(const Gpd32Args& A, const Sp32& S, int32_t* slots, const int rel[3],
                                             int32_t gcell) {
    int sl = 0, mul = 1;
    bool win = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int e = A.sext[d];
        const int x = e == 1 ? 0 : rel[d] + 2;
        win = win && x >= 0 && x < e;
        sl += x * mul;
        mul *= e;
    }
    if (win) {
        const int32_t r = atomicAdd(&slots[sl], 1);
        if (r < (1 << 20)) return (sl << 20) | r;
    }
    return (int32_t)(0x80000000u | (uint32_t)atomicAdd(&S.cnt[gcell], 1));
}

// What the charge-conserving deposit of one particle needs, kept in registers between its step
// and its deposit: the old offset, the new position relative to the old cell and the cell's
// place in the tile (the window is built from them at deposit time).
template <int O>
struct Win {
    float f[3], x1[3];
    int loc[3];
    bool dep;
};

// The Esirkepov window of a particle: S0 and DS = S1 - S0 on the O + 2 centred nodes per axis
// covering the old and the new support, the window's first node in the tile's current block,
// and which axes the supports differ on.
template <int O, class TL>
__device__ __forceinline__ void make_window(const TL& L, const Win<O>& W, float S0[3][O + 2], float DS[3][O + 2],
                                            int wb[3], int& moved) {
    const int clo[3] = {L.clox, L.cloy, L.cloz};
    moved = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float w0[O + 1], w1[O + 1];
        const int a0 = centred_weights<O>(W.f[d], w0);
        const int a1 = centred_weights<O>(W.x1[d], w1);
        const bool lo1 = a1 < a0;  // the new support starts one node lower
        const bool hi1 = a1 > a0;
        const int bmin = lo1 ? a1 : a0;
#pragma unroll
        for (int kk = 0; kk < O + 2; ++kk) {
            // old weights sit at window offset (a0 - bmin), new at (a1 - bmin)
            const float s0 = lo1 ? (kk >= 1 ? w0[kk - 1 < O ? kk - 1 : O] : 0.f) : (kk <= O ? w0[kk <= O ? kk : O] : 0.f);
            const float s1 = hi1 ? (kk >= 1 ? w1[kk - 1 < O ? kk - 1 : O] : 0.f) : (kk <= O ? w1[kk <= O ? kk : O] : 0.f);
            S0[d][kk] = s0;
            DS[d][kk] = s1 - s0;
        }
        wb[d] = W.loc[d] + clo[d] + bmin;
        moved |= (lo1 || hi1) ? 1 << d : 0;
    }
}

// First node of a particle's window along axis d (as make_window), without the weights.
template <int O, class TL>
__device__ __forceinline__ int window_start(const TL& L, const Win<O>& W, int d) {
    const int clo[3] = {L.clox, L.cloy, L.cloz};
    const int a0 = O == 2 ? (int)floorf(W.f[d] + 0.5f) - 1 : (int)floorf(W.f[d]) - 1;
    const int a1 = O == 2 ? (int)floorf(W.x1[d] + 0.5f) - 1 : (int)floorf(W.x1[d]) - 1;
    return W.loc[d] + clo[d] + (a1 < a0 ? a1 : a0);
}

// What the particle step of one tile and species needs besides the arguments.
struct TileCtx {
    int org[3];
    int64_t base_cell;
    int nxy;
    const float* fld;
    unsigned long long* cur;
    int32_t* slots;
    double facq[3];  // -q w d_c / dt, times the fixed-point scale
    double qwq;      // q w times the fixed-point scale (direct current)
};

// The particle step of slot q (gather, push, move, renormalise, store, rank for the next sort;
// the direct current is deposited here).  For the charge-conserving current the window is left
// in W for the deposit (W.dep = false when the particle deposits nothing: left as it was, or
// the direct scheme).
template <int O, class TL>
__device__ __forceinline__ void step_particle(const Gpd32Args& A, const Sp32& S, const TL& L, const TileCtx& C,
                                              int32_t q, Win<O>& W, int& bad_all) {
    W.dep = false;
    const int n0 = A.n[0], n1 = A.n[1], n2 = A.n[2];
    const int32_t p = S.perm ? S.perm[q] : q;
    if (p < 0) {  // an empty slot (counts made inconsistent by flagged particles)
        S.rank[q] = -1;
        return;
    }
    const int32_t cell = S.cell[p];
    float f[3] = {S.pos[0][p], S.pos[1][p], S.pos[2][p]};
    V3<float> u{S.u[0][p], S.u[1][p], S.u[2][p]};
    if (S.id) S.id_o[q] = S.id[p];
    // a particle left as it is still moves to its slot when the kernel reorders
    auto keep = [&](const V3<float>& uk) {
        if (!S.perm) return;
        S.cell_o[q] = cell;
        S.pos_o[0][q] = f[0];
        S.pos_o[1][q] = f[1];
        S.pos_o[2][q] = f[2];
        S.u_o[0][q] = uk.x;
        S.u_o[1][q] = uk.y;
        S.u_o[2][q] = uk.z;
    };
    // position inside the tile: rel = li + n0 lj + n0 n1 lk with l < t, found by
    // comparisons (no division)
    int64_t rel = (int64_t)cell - C.base_cell;
    int lk = 0, lj = 0;
    while (lk < L.tz - 1 && rel >= (int64_t)C.nxy) {
        rel -= C.nxy;
        ++lk;
    }
    while (lj < L.ty - 1 && rel >= (int64_t)n0) {
        rel -= n0;
        ++lj;
    }
    const int li = (int)rel;
    const int loc[3] = {li, lj, lk};
    const int* org = C.org;
    // the particle must lie in this tile: local indices in range and the cell index
    // rebuilt from them equal to the stored one
    const bool inside = rel >= 0 && li < L.tx && org[0] + li < n0 && org[1] + lj < n1 && org[2] + lk < n2 &&
                        (int64_t)(org[0] + li) + (int64_t)n0 * ((org[1] + lj) + (int64_t)n1 * (org[2] + lk)) ==
                            (int64_t)cell;
    if (!inside) {  // not this tile's particle: left out of the next sort
        bad_all |= PP_FLAG_OUT_OF_TILE;
        keep(u);
        S.rank[q] = -1;
        return;
    }
    if (!offset_ok<O>(f[0]) || !offset_ok<O>(f[1]) || !offset_ok<O>(f[2])) {  // left as it is
        bad_all |= PP_FLAG_OUT_OF_TILE;
        keep(u);
        S.rank[q] = dest_rank(A, S, C.slots, loc, cell);
        return;
    }

    // gather (eq. "pfields") from the LDS field tile
    float wc[3][O + 1], ws[3][O + 1];
    int fc[3], fs[3];
    {
        const int flo[3] = {L.flox, L.floy, L.floz};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int bc, bs;
            split_weights<O>(f[d], wc[d], bc, ws[d], bs);
            fc[d] = loc[d] + flo[d] + bc;
            fs[d] = loc[d] + flo[d] + bs;
        }
    }
    const float* fld = C.fld;
    V3<float> E, B;
    E.x = gather_comp<O>(fld + 0 * L.fvol, L, fs[0], fc[1], fc[2], ws[0], wc[1], wc[2]);
    E.y = gather_comp<O>(fld + 1 * L.fvol, L, fc[0], fs[1], fc[2], wc[0], ws[1], wc[2]);
    E.z = gather_comp<O>(fld + 2 * L.fvol, L, fc[0], fc[1], fs[2], wc[0], wc[1], ws[2]);
    B.x = gather_comp<O>(fld + 3 * L.fvol, L, fc[0], fs[1], fs[2], wc[0], ws[1], ws[2]);
    B.y = gather_comp<O>(fld + 4 * L.fvol, L, fs[0], fc[1], fs[2], ws[0], wc[1], ws[2]);
    B.z = gather_comp<O>(fld + 5 * L.fvol, L, fs[0], fs[1], fc[2], ws[0], ws[1], wc[2]);

    const V3<float> um = u;
    if (A.pusher == PP_PUSH_BORIS)
        push_boris<float>(S.h, A.ic, E, B, u);
    else
        push_vay<float>(S.h, A.ic, E, B, u);
    if (S.krad != 0.0f) rad_cool<float>(S.krad, A.dtk, A.ic, um, u);

    const float ig = rsqrtf(1.0f + dot(u, u) * A.ic * A.ic);
    const float uu[3] = {u.x, u.y, u.z};
    float x1[3], dxs[3];
    int bad = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float dd = A.dt * uu[d] * ig * A.inv_d[d];
        if (!(fabsf(dd) < 1.0f)) bad |= isfinite(dd) ? PP_FLAG_CFL : PP_FLAG_NONFINITE;
        if (!isfinite(uu[d])) bad |= PP_FLAG_NONFINITE;
        x1[d] = f[d] + dd;  // new position relative to the old cell's node
        dxs[d] = dd;
    }
    if (bad) {  // left as it was before the push
        bad_all |= bad;
        keep(um);
        S.rank[q] = dest_rank(A, S, C.slots, loc, cell);
        return;
    }

    if (A.direct) {
        // direct current (eq. "jj2"): q w v_c W at J_c's staggered nodes, at the
        // time-centred offset f + dd/2 (its supports stay inside the block's halo)
        float wcm[3][O + 1], wsm[3][O + 1];
        int ncm[3], nsm[3];
        const int clo[3] = {L.clox, L.cloy, L.cloz};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int bc, bs;
            split_weights<O>(f[d] + 0.5f * dxs[d], wcm[d], bc, wsm[d], bs);
            ncm[d] = loc[d] + clo[d] + bc;
            nsm[d] = loc[d] + clo[d] + bs;
        }
        const int cst[3] = {L.csx, L.csy, L.csz};
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) {
            unsigned long long* Jc = C.cur + comp * L.cvol;
            const double vq = C.qwq * (double)(uu[comp] * ig);
            const int n0x = comp == 0 ? nsm[0] : ncm[0];
            const int n0y = comp == 1 ? nsm[1] : ncm[1];
            const int n0z = comp == 2 ? nsm[2] : ncm[2];
            const float* wx = comp == 0 ? wsm[0] : wcm[0];
            const float* wy = comp == 1 ? wsm[1] : wcm[1];
            const float* wz = comp == 2 ? wsm[2] : wcm[2];
#pragma unroll
            for (int c = 0; c <= O; ++c) {
#pragma unroll
                for (int b = 0; b <= O; ++b) {
                    const double wzy = vq * (double)(wz[c] * wy[b]);
                    const int rowo = n0x * cst[0] + (n0y + b) * cst[1] + (n0z + c) * cst[2];
#pragma unroll
                    for (int a = 0; a <= O; ++a) {
                        const double dq = fma(wzy, (double)wx[a], ROUND_MAGIC);
                        atomicAdd(Jc + rowo + a * cst[0], (unsigned long long)__double_as_longlong(dq));
                    }
                }
            }
        }
    } else {
        // the charge-conserving current is deposited later, from these
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            W.f[d] = f[d];
            W.x1[d] = x1[d];
            W.loc[d] = loc[d];
        }
        W.dep = true;
    }

    // renormalise: new cell and offset in [lo, lo + 1), or in [lo + 1, lo + 2) in the
    // cell below when the next displacement (this one times the ratio of the next drift
    // to this one) would cross the lower face
    int nc3[3], shv[3];
    float fn[3];
    const int gc[3] = {org[0] + li, org[1] + lj, org[2] + lk};
    const float lo = off_lo<O>();
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float sh = floorf(x1[d] - lo);
        float o = x1[d] - sh;
        // rounding can land the offset just outside the range: move it back in
        if (o < lo) {
            o += 1.0f;
            sh -= 1.0f;
        } else if (o >= lo + 1.0f) {
            o -= 1.0f;
            sh += 1.0f;
        }
        const float up = o + 1.0f;
        if (o + dxs[d] * A.pred < lo && up < lo + 2.0f) {
            o = up;
            sh -= 1.0f;
        }
        fn[d] = o;
        shv[d] = (int)sh;
        nc3[d] = wrap_near(gc[d] + (int)sh, A.n[d]);
    }
    const int32_t newcell = nc3[0] + n0 * (nc3[1] + n1 * nc3[2]);
    S.cell_o[q] = newcell;
    S.pos_o[0][q] = fn[0];
    S.pos_o[1][q] = fn[1];
    S.pos_o[2][q] = fn[2];
    S.u_o[0][q] = u.x;
    S.u_o[1][q] = u.y;
    S.u_o[2][q] = u.z;
    const int dst[3] = {li + shv[0], lj + shv[1], lk + shv[2]};
    S.rank[q] = dest_rank(A, S, C.slots, dst, newcell);
}

// Charge-conserving current of one particle (W1), or of two particles whose windows start at
// the same node of the block (W1 and W2, PAIR): per component the prefix sums of DS along the
// component's axis times the scaled factor, P_a, and for every transverse node pair the
// factor F = S0_1 (S0_2 + DS_2/2) + DS_1 (S0_2/2 + DS_2/3); each node then receives the bits
// of (1.5*2^52 + round(P_a F)) in one 64-bit integer atomic.  For a pair the two patterns,
// each rounded on its own, are added as integers before the one atomic, so the node gets the
// same exact fixed-point sum as from two atomics.  f2 != 0 marks lanes whose second particle
// deposits; on the others its prefix sums are zeros, so that its patterns are 1.5*2^52 itself,
// whose low 51 bits are zero (the caller keeps that particle's window state finite).
template <int O, class TL, bool PAIR>
__device__ __forceinline__ void deposit_cc(const TL& L, unsigned long long* cur, const Win<O>& P1, const double* facq1,
                                           const Win<O>& P2, const double* facq2, float f2) {
    float S0a[3][O + 2], DSa[3][O + 2], S0b[3][O + 2], DSb[3][O + 2];
    int wb[3], wb2[3], moved1, moved2 = 0;
    make_window<O, TL>(L, P1, S0a, DSa, wb, moved1);
    if (PAIR) make_window<O, TL>(L, P2, S0b, DSb, wb2, moved2);
    struct WinF {
        const float (*S0)[O + 2];
        const float (*DS)[O + 2];
    } W1{S0a, DSa}, W2{S0b, DSb};
    const int cst[3] = {L.csx, L.csy, L.csz};
    const bool use2 = PAIR && f2 != 0.0f;
    const int moved = use2 ? (moved1 | moved2) : moved1;
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        const int d1 = comp == 0 ? 1 : (comp == 1 ? 2 : 0);
        const int d2 = comp == 0 ? 2 : (comp == 1 ? 0 : 1);
        unsigned long long* Jc = cur + comp * L.cvol;
        const int off0 = wb[0] * L.csx + wb[1] * L.csy + wb[2] * L.csz;
        // prefix sums of DS along the component's own axis (the last one vanishes),
        // scaled to fixed-point units: P_a * fac * 2^e in FP64
        // A particle whose supports coincide along the component's axis contributes nothing
        // at the last node even when its partner's does: its last prefix sum is only the
        // rounding residue of a vanishing sum, which the single deposit leaves out too.
        const bool own1 = (moved1 >> comp) & 1, own2 = (moved2 >> comp) & 1;
        double Pq1[O + 1], Pq2[O + 1];
        float acc1 = 0.f, acc2 = 0.f;
#pragma unroll
        for (int a = 0; a <= O; ++a) {
            acc1 += W1.DS[comp][a];
            Pq1[a] = (a < O || own1) ? (double)acc1 * facq1[comp] : 0.0;
            if (PAIR) {  // zero for a second particle that deposits nothing
                acc2 += W2.DS[comp][a];
                Pq2[a] = (use2 && (a < O || own2)) ? (double)acc2 * facq2[comp] : 0.0;
            }
        }
        const bool m1 = (moved >> d1) & 1, m2 = (moved >> d2) & 1, mc = (moved >> comp) & 1;
        // Along an axis where the supports coincide the window's last node carries no
        // weight (its transverse factors are exactly zero) and the last prefix sum is
        // the rounding residue of a vanishing sum: those additions are left out.
#pragma unroll
        for (int bq = 0; bq < O + 2; ++bq) {
            if (bq == O + 1 && !m1) continue;
            const float g1 = W1.S0[d1][bq], h1 = W1.DS[d1][bq];
            const float g2 = PAIR ? W2.S0[d1][bq] : 0.f, h2 = PAIR ? W2.DS[d1][bq] : 0.f;
#pragma unroll
            for (int e = 0; e < O + 2; ++e) {
                if (e == O + 1 && !m2) continue;
                const double Fd1 = (double)(g1 * (W1.S0[d2][e] + 0.5f * W1.DS[d2][e]) +
                                            h1 * (0.5f * W1.S0[d2][e] + (1.0f / 3.0f) * W1.DS[d2][e]));
                double Fd2 = 0.0;
                if (PAIR)
                    Fd2 = (double)(g2 * (W2.S0[d2][e] + 0.5f * W2.DS[d2][e]) +
                                   h2 * (0.5f * W2.S0[d2][e] + (1.0f / 3.0f) * W2.DS[d2][e]));
                const int rowo = off0 + bq * cst[d1] + e * cst[d2];
#pragma unroll
                for (int a = 0; a <= O; ++a) {
                    if (a == O && !mc) continue;
                    // bits of (1.5*2^52 + round(P_a F fac 2^e)): see the header.  A pair
                    // adds its two patterns as integers: each contribution is rounded on its
                    // own, as by two atomics (a chained FMA would round the second one
                    // against the first, and a tie could then round the other way).
                    unsigned long long bits = (unsigned long long)__double_as_longlong(fma(Pq1[a], Fd1, ROUND_MAGIC));
                    if (PAIR) bits += (unsigned long long)__double_as_longlong(fma(Pq2[a], Fd2, ROUND_MAGIC));
                    atomicAdd(Jc + rowo + a * cst[comp], bits);
                }
            }
        }
    }
}

// One tile of one run: the whole particle step of the tile's particles (the body shared by
// the single-run kernel and the batched kernel, so both do identical arithmetic).
// Each wavefront takes 128 consecutive slots at a time, lane l the slots l and 64 + l.  In
// the chunks of pairs of the tile order both are a particle of the same cell, whose current
// windows start at the same node unless one of the particles crossed a face the storage did
// not expect; such pairs deposit together with one atomic per node for both.  Where some
// lane's pair does not share a window, that lane's second particle deposits alone in a second
// pass; where no lane's does (the single particles after the chunks), each particle deposits
// alone.  Flat (8x8x1) and runtime-shaped tiles take one particle per lane and slot (64
// consecutive slots per wavefront).
template <int O, class TL>
__device__ __forceinline__ void gpd32_tile(const Gpd32Args& A, int64_t tile, unsigned char* lds_raw) {
    const TL L(A);
    const int ti = (int)(tile % A.nt[0]);
    const int tj = (int)((tile / A.nt[0]) % A.nt[1]);
    const int tk = (int)(tile / ((int64_t)A.nt[0] * A.nt[1]));
    const int org[3] = {ti * L.tx, tj * L.ty, tk * L.tz};
    const int n0 = A.n[0], n1 = A.n[1], n2 = A.n[2];

    // fields first: the gather's LDS reads then use small immediate offsets
    float* fld = (float*)lds_raw;  // 6 * fvol
    unsigned long long* cur = (unsigned long long*)(lds_raw + ((6 * L.fvol * sizeof(float) + 15) & ~(size_t)15));

    // 1. stage fields (each thread has STAGE_BATCH loads in flight before it waits for the
    // first), clear the current block
    for (int q0 = threadIdx.x; q0 < 6 * L.fvol; q0 += STAGE_BATCH * GPD32_BS) {
        double v[STAGE_BATCH];
        int dst[STAGE_BATCH];  // LDS entry, or -1 (past the end, or padding)
#pragma unroll
        for (int k = 0; k < STAGE_BATCH; ++k) {
            // every lane loads (an entry past the end or in the padding reads a node of the
            // tile instead and writes nothing), so that no load waits at a branch
            const int q = q0 + k * GPD32_BS;
            const int qc = q < 6 * L.fvol ? q : 0;
            const int comp = qc / L.fvol;
            const int r = qc - comp * L.fvol;
            const int c = r / L.fplane;
            const int rr = r - c * L.fplane;
            const int bb = rr / L.frow;
            const int a = rr - bb * L.frow;
            dst[k] = (q < 6 * L.fvol && a < L.fex && bb < L.fey) ? q : -1;
            const int gi = wrap_near(org[0] - L.flox + (a < L.fex ? a : 0), n0);
            const int gj = wrap_near(org[1] - L.floy + (bb < L.fey ? bb : 0), n1);
            const int gk = wrap_near(org[2] - L.floz + c, n2);
            const int64_t gq = (int64_t)gi + (int64_t)n0 * (gj + (int64_t)n1 * gk);
            const double* src = comp < 3 ? A.E + comp * A.nc : A.B + (comp - 3) * A.nc;
            v[k] = src[gq];
        }
#pragma unroll
        for (int k = 0; k < STAGE_BATCH; ++k)
            if (dst[k] >= 0) fld[dst[k]] = (float)v[k];
    }
    for (int q = threadIdx.x; q < 3 * L.cvol; q += GPD32_BS) cur[q] = 0ull;
    int32_t* slots = (int32_t*)(cur + 3 * L.cvol);  // A.nslots destination-cell counters
    for (int q = threadIdx.x; q < A.nslots; q += GPD32_BS) slots[q] = 0;
    __syncthreads();

    TileCtx C;
    for (int d = 0; d < 3; ++d) C.org[d] = org[d];
    C.base_cell = (int64_t)org[0] + (int64_t)n0 * (org[1] + (int64_t)n1 * org[2]);
    C.nxy = n0 * n1;
    C.fld = fld;
    C.cur = cur;
    C.slots = slots;
    const double qs = *A.qscale;
    int bad_all = 0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

    for (int s = 0; s < A.nsp; ++s) {
        const Sp32& S = A.sp[s];
        const int32_t start = S.start[tile];
        const int32_t end = S.start[tile + 1];
        for (int d = 0; d < 3; ++d) C.facq[d] = S.fac[d] * qs;
        C.qwq = S.qw * qs;
        if constexpr (!TL::pairs) {
            for (int32_t q = start + threadIdx.x; q < end; q += GPD32_BS) {
                Win<O> W;
                step_particle<O, TL>(A, S, L, C, q, W, bad_all);
                if (W.dep) deposit_cc<O, TL, false>(L, cur, W, C.facq, W, C.facq, 0.0f);
            }
        } else {
            for (int32_t b = start + 128 * wave; b < end; b += 4 * 128) {
                Win<O> W1, W2;
                const int32_t q1 = b + lane, q2 = b + 64 + lane;
                W1.dep = W2.dep = false;
                // a second particle that deposits nothing still enters the paired deposit with
                // zero prefix sums: its window state must then be finite
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    W2.f[d] = W2.x1[d] = 0.5f;
                    W2.loc[d] = 0;
                }
                if (q1 < end) step_particle<O, TL>(A, S, L, C, q1, W1, bad_all);
                if (q2 < end) step_particle<O, TL>(A, S, L, C, q2, W2, bad_all);
                const bool both = W1.dep && W2.dep;
                const bool same = both && window_start<O, TL>(L, W1, 0) == window_start<O, TL>(L, W2, 0) &&
                                  window_start<O, TL>(L, W1, 1) == window_start<O, TL>(L, W2, 1) &&
                                  window_start<O, TL>(L, W1, 2) == window_start<O, TL>(L, W2, 2);
                if (__any(same)) {
                    // the first particle of every lane (or its second, if only that one deposits),
                    // together with the second where the windows coincide
                    if (!W1.dep && W2.dep) {
                        W1 = W2;
                        W2.dep = false;
                    }
                    if (W1.dep)
                        deposit_cc<O, TL, true>(L, cur, W1, C.facq, W2, C.facq, same ? 1.0f : 0.0f);
                    if (both && !same) deposit_cc<O, TL, false>(L, cur, W2, C.facq, W2, C.facq, 0.0f);
                } else {
                    if (W1.dep) deposit_cc<O, TL, false>(L, cur, W1, C.facq, W1, C.facq, 0.0f);
                    if (W2.dep) deposit_cc<O, TL, false>(L, cur, W2, C.facq, W2, C.facq, 0.0f);
                }
            }
        }
        // reserve the tile's range in each destination cell's count, then complete the ranks
        __syncthreads();
        for (int q = threadIdx.x; q < A.nslots; q += GPD32_BS) {
            const int c = slots[q];
            if (c == 0) continue;
            const int x = q % A.sext[0], y = (q / A.sext[0]) % A.sext[1], z = q / (A.sext[0] * A.sext[1]);
            const int gx = A.sext[0] == 1 ? 0 : wrap(org[0] + x - 2, n0);
            const int gy = A.sext[1] == 1 ? 0 : wrap(org[1] + y - 2, n1);
            const int gz = A.sext[2] == 1 ? 0 : wrap(org[2] + z - 2, n2);
            slots[q] = atomicAdd(&S.cnt[gx + n0 * (gy + n1 * gz)], c);
        }
        __syncthreads();
        for (int32_t p = start + threadIdx.x; p < end; p += GPD32_BS) {
            const int32_t v = S.rank[p];
            if (v == -1) continue;
            S.rank[p] = v < 0 ? (v & 0x7FFFFFFF) : slots[v >> 20] + (v & 0xFFFFF);
        }
        __syncthreads();
        for (int q = threadIdx.x; q < A.nslots; q += GPD32_BS) slots[q] = 0;
        __syncthreads();
    }
    if (bad_all) atomic_or_flag(A.flags, bad_all);

    // 3. flush the current block (integer adds commute: the sum is order-independent); each
    // thread reads STAGE_BATCH entries before it waits for the first
    for (int q0 = threadIdx.x; q0 < 3 * L.cvol; q0 += STAGE_BATCH * GPD32_BS) {
        unsigned long long raw[STAGE_BATCH];
#pragma unroll
        for (int k = 0; k < STAGE_BATCH; ++k) {
            const int q = q0 + k * GPD32_BS;
            raw[k] = q < 3 * L.cvol ? cur[q] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < STAGE_BATCH; ++k) {
            const int q = q0 + k * GPD32_BS;
            const long long v = fixed_sum(raw[k]);
            if (v == 0) continue;  // also every entry past the end
            const int comp = q / L.cvol;
            const int r = q - comp * L.cvol;
            const int c = r / L.cplane;
            const int rr = r - c * L.cplane;
            const int bb = rr / L.crow;
            const int a = rr - bb * L.crow;
            if (bb >= L.cey) continue;  // padding
            const int gi = wrap_near(org[0] - L.clox + a, n0);
            const int gj = wrap_near(org[1] - L.cloy + bb, n1);
            const int gk = wrap_near(org[2] - L.cloz + c, n2);
            atomicAdd(A.Jq + comp * A.nc + (int64_t)gi + (int64_t)n0 * (gj + (int64_t)n1 * gk),
                      (unsigned long long)v);
        }
    }
}

template <int O, class TL>
__global__ void __launch_bounds__(GPD32_BS, TL::pairs ? 3 : 1) k_gpd32(Gpd32Args A) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    // XCD-aware tile order: consecutive workgroups go round-robin over the 8 XCDs, so give
    // each XCD a contiguous run of tiles (neighbouring tiles share halos in that XCD's L2).
    const int64_t b = blockIdx.x;
    const int64_t tile = (b & 7) * (int64_t)A.per_xcd + (b >> 3);
    if (tile >= A.ntiles) return;
    gpd32_tile<O, TL>(A, tile, lds_raw);
}

// Batched: block b of the launch is tile b - prefix[r] of run r (prefix = running tile counts).
template <int O, class TL>
__global__ void __launch_bounds__(GPD32_BS, TL::pairs ? 3 : 1) k_gpd32_batch(const Gpd32Args* __restrict__ table,
                                                          const int64_t* __restrict__ prefix, int nruns) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int64_t b = blockIdx.x;
    const int r = find_segment(prefix, nruns, b);
    if (r < 0) return;
    gpd32_tile<O, TL>(table[r], b - prefix[r], lds_raw);
}

// Fixed-point current bookkeeping of one run: scale, accumulator, FP64 target.
struct FixedDesc {
    const int32_t* tile_max;  // largest tile population per species slot
    int e0;                   // host part of the exponent
    double* scale;            // 2^e (device)
    unsigned long long* Jq;   // accumulator, 3 * nc
    double* J;                // FP64 current written from the accumulator
    int64_t n3;
};

// 2^e with e = e0 - ceil(log2(N)), N the sum over species of the largest particle count of
// any tile: then |one contribution| <= 2^(50 - ceil log2 N) and |a node's LDS sum| <= 2^50.
__device__ __forceinline__ void fixed_scale_body(const FixedDesc& D) {
    long long nb = 0;
    for (int s = 0; s < PP_MAX_SPECIES; ++s) nb += D.tile_max[s];
    int lg = 0;
    while ((1ll << lg) < nb) ++lg;
    *D.scale = ldexp(1.0, D.e0 - lg);
}

enum FixedPhase { FX_ZERO = 0, FX_TO_F64 = 1 };

__device__ __forceinline__ void fixed_body(const FixedDesc& D, int64_t q, int phase) {
    if (q >= D.n3) return;
    if (phase == FX_ZERO) {
        D.Jq[q] = 0ull;
    } else {
        const double inv = 1.0 / *D.scale;  // exact: a power of two
        D.J[q] = (double)(long long)D.Jq[q] * inv;
    }
}

__global__ void k_fixed_scale(FixedDesc D) {
    if (blockIdx.x == 0 && threadIdx.x == 0) fixed_scale_body(D);
}

__global__ void __launch_bounds__(256) k_fixed(FixedDesc D, int phase) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < D.n3; q += (int64_t)gridDim.x * blockDim.x)
        fixed_body(D, q, phase);
}

__global__ void k_fixed_scale_batch(const FixedDesc* __restrict__ T, int n) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) fixed_scale_body(T[r]);
}

__global__ void __launch_bounds__(256) k_fixed_batch(const FixedDesc* __restrict__ T, const int64_t* __restrict__ prefix,
                                                     int n, int phase) {
    const int64_t b = blockIdx.x;
    const int r = find_segment(prefix, n, b);
    if (r < 0) return;
    fixed_body(T[r], (b - prefix[r]) * blockDim.x + threadIdx.x, phase);
}

enum TileKind { TILE_444 = 0, TILE_881_FLAT = 1, TILE_RT = 2 };

static int tile_kind(const pp_run* r) {
    const int* t = r->g.t;
    const int* n = r->p.n;
    if (t[0] == 4 && t[1] == 4 && t[2] == 4 && n[0] > 1 && n[1] > 1 && n[2] > 1) return TILE_444;
    if (t[0] == 8 && t[1] == 8 && t[2] == 1 && n[0] > 1 && n[1] > 1 && n[2] == 1) return TILE_881_FLAT;
    return TILE_RT;
}

static void lds_extents(const pp_run* r, int fe[3], int ce[3], int flo[3], int clo[3]) {
    for (int d = 0; d < 3; ++d) {
        const bool single = r->p.n[d] == 1;
        fe[d] = single ? 1 : r->g.t[d] + FLD_LO + fld_hi(r->p.shape_order);
        ce[d] = single ? 1 : r->g.t[d] + cur_lo(r->p.shape_order) + cur_hi(r->p.shape_order);
        flo[d] = single ? 0 : FLD_LO;
        clo[d] = single ? 0 : cur_lo(r->p.shape_order);
    }
}

size_t gpd32_lds_bytes(const pp_run* r) {
    int fe[3], ce[3], flo[3], clo[3];
    lds_extents(r, fe, ce, flo, clo);
    const size_t fv = tile_kind(r) == TILE_444 ? (size_t)fld_plane_444(r->p.shape_order) * fe[2]
                                                : (size_t)fe[0] * fe[1] * fe[2];
    const int kind = tile_kind(r);
    const size_t cv = kind == TILE_444       ? (size_t)cur_plane_444(r->p.shape_order) * ce[2]
                      : kind == TILE_881_FLAT ? (size_t)cur_row_881 * ce[1]
                                              : (size_t)ce[0] * ce[1] * ce[2];
    size_t slots = 1;
    for (int d = 0; d < 3; ++d) slots *= r->p.n[d] == 1 ? 1 : (size_t)r->g.t[d] + 4;
    return ((6 * fv * sizeof(float) + 15) & ~(size_t)15) + 3 * cv * sizeof(unsigned long long) + slots * sizeof(int32_t);
}

// Host part of the fixed-point exponent: e0 = 50 - ceil(log2(max |fac|)), every contribution
// being at most |fac| = |q w d / dt| in magnitude (|prefix of DS| <= 1 and 0 <= F <= 1).
int gpd32_scale_e0(const pp_run* r) {
    double fmax = 0.0;
    for (int s = 0; s < PP_MAX_SPECIES; ++s) {
        const Species& S = r->sp[s];
        if (!S.active) continue;
        for (int d = 0; d < 3; ++d) {
            const double f = fabs(S.q * S.w * r->p.d[d] / r->dt_drift);
            fmax = f > fmax ? f : fmax;
        }
    }
    if (!(fmax > 0.0)) return 0;
    // on a single-cell axis the O+2 window nodes of a particle all land on one LDS node, so a
    // node can receive up to O+2 contributions of one particle per such axis
    int collapsed = 0;
    for (int d = 0; d < 3; ++d) collapsed += r->p.n[d] == 1 ? 1 : 0;
    const int per_axis = (int)ceil(log2((double)(r->p.shape_order + 2)));
    return 50 - (int)ceil(log2(fmax)) - collapsed * per_axis;
}

// Kernel arguments of one run (also the batched table entries).
void gpd32_fill_args(const pp_run* r, Gpd32Args* Ap) {
    Gpd32Args& A = *Ap;
    int fe[3], ce[3], flo[3], clo[3];
    lds_extents(r, fe, ce, flo, clo);
    for (int d = 0; d < 3; ++d) {
        A.n[d] = r->p.n[d];
        A.t[d] = r->g.t[d];
        A.nt[d] = r->g.nt[d];
        A.fe[d] = fe[d];
        A.ce[d] = ce[d];
        A.flo[d] = flo[d];
        A.clo[d] = clo[d];
        A.inv_d[d] = (float)(1.0 / r->p.d[d]);
    }
    A.ntiles = r->g.ntiles;
    A.nc = r->g.ncell;
    A.dt = (float)r->dt_drift;
    A.dtk = (float)r->dt_kick;
    A.pred = (float)r->drift_ratio;
    A.ic = (float)(1.0 / r->p.c);
    A.pusher = r->p.pusher;
    A.nsp = 0;
    for (int s = 0; s < PP_MAX_SPECIES; ++s) {
        const Species& S = r->sp[s];
        if (!S.active) continue;
        Sp32& D = A.sp[A.nsp++];
        D.start = S.offsets;
        D.cnt = S.cell_cnt;
        D.rank = S.rank;
        D.perm = S.pending ? S.perm : nullptr;
        D.cell = S.cur.cell;
        D.cell_o = S.pending ? S.cur.cell_alt : S.cur.cell;
        D.id = S.pending ? S.cur.id : nullptr;
        D.id_o = S.pending ? S.cur.id_alt : nullptr;
        for (int d = 0; d < 3; ++d) {
            D.pos[d] = (const float*)S.cur.pos[d];
            D.u[d] = (const float*)S.cur.u[d];
            D.pos_o[d] = (float*)(S.pending ? S.cur.pos_alt[d] : S.cur.pos[d]);
            D.u_o[d] = (float*)(S.pending ? S.cur.u_alt[d] : S.cur.u[d]);
            D.fac[d] = -S.q * S.w * r->p.d[d] / r->dt_drift;
        }
        D.h = (float)(S.q * r->dt_kick / S.m);
        D.krad = (float)(r->p.rad_tau * S.q * S.q / S.m);
        D.qw = S.q * S.w;
    }
    A.E = r->mesh.E;
    A.B = r->mesh.B;
    A.Jq = (unsigned long long*)r->Jq;
    A.qscale = r->qscale;
    A.flags = r->flags;
    A.per_xcd = (int)((r->g.ntiles + 7) / 8);
    A.direct = r->p.current_scheme == PP_CURRENT_DIRECT ? 1 : 0;
    A.nslots = 1;
    for (int d = 0; d < 3; ++d) {
        A.sext[d] = r->p.n[d] == 1 ? 1 : r->g.t[d] + 4;
        A.nslots *= A.sext[d];
    }
}

void gpd32_fixed_desc(const pp_run* r, double* J, FixedDesc* D) {
    D->tile_max = r->tile_max;
    D->e0 = gpd32_scale_e0(r);
    D->scale = r->qscale;
    D->Jq = (unsigned long long*)r->Jq;
    D->J = J;
    D->n3 = 3 * r->g.ncell;
}

size_t gpd32_args_size() { return sizeof(Gpd32Args); }
size_t gpd32_fixed_desc_size() { return sizeof(FixedDesc); }
bool gpd32_batchable(const pp_run* r) { return tile_kind(r) == TILE_444; }

static unsigned fixed_grid(int64_t n3) {
    int64_t g = (n3 + 255) / 256;
    if (g > 16384) g = 16384;
    return (unsigned)(g < 1 ? 1 : g);
}

hipError_t launch_gpd32(pp_run* r, double* J) {
    Gpd32Args A;
    gpd32_fill_args(r, &A);
    FixedDesc F;
    gpd32_fixed_desc(r, J, &F);
    hipLaunchKernelGGL(k_fixed_scale, dim3(1), dim3(64), 0, r->stream, F);
    hipLaunchKernelGGL(k_fixed, dim3(fixed_grid(F.n3)), dim3(256), 0, r->stream, F, (int)FX_ZERO);
    const size_t lds = gpd32_lds_bytes(r);
    const unsigned grid = (unsigned)(8 * (int64_t)A.per_xcd);
    const int kind = tile_kind(r);
    if (r->p.shape_order == 2) {
        if (kind == TILE_444)
            hipLaunchKernelGGL((k_gpd32<2, TileCT<2, 4, 4, 4, false>>), dim3(grid), dim3(GPD32_BS), lds, r->stream, A);
        else if (kind == TILE_881_FLAT)
            hipLaunchKernelGGL((k_gpd32<2, TileCT<2, 8, 8, 1, true>>), dim3(grid), dim3(GPD32_BS), lds, r->stream, A);
        else
            hipLaunchKernelGGL((k_gpd32<2, TileRT>), dim3(grid), dim3(GPD32_BS), lds, r->stream, A);
    } else {
        if (kind == TILE_444)
            hipLaunchKernelGGL((k_gpd32<3, TileCT<3, 4, 4, 4, false>>), dim3(grid), dim3(GPD32_BS), lds, r->stream, A);
        else if (kind == TILE_881_FLAT)
            hipLaunchKernelGGL((k_gpd32<3, TileCT<3, 8, 8, 1, true>>), dim3(grid), dim3(GPD32_BS), lds, r->stream, A);
        else
            hipLaunchKernelGGL((k_gpd32<3, TileRT>), dim3(grid), dim3(GPD32_BS), lds, r->stream, A);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (J) hipLaunchKernelGGL(k_fixed, dim3(fixed_grid(F.n3)), dim3(256), 0, r->stream, F, (int)FX_TO_F64);
    return hipGetLastError();
}

// Batched particle step of n runs that all use 4x4x4 tiles and the same weight order:
// fixed-point scales, accumulator clear, the tiled kernel, conversion to FP64.
hipError_t launch_gpd32_batch(const void* args_table, const int64_t* tile_prefix, int64_t total_tiles,
                              const void* fixed_table, const int64_t* fixed_prefix, int64_t total_fixed_blocks, int n,
                              int shape_order, size_t lds, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const FixedDesc* F = (const FixedDesc*)fixed_table;
    hipLaunchKernelGGL(k_fixed_scale_batch, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, F, n);
    hipLaunchKernelGGL(k_fixed_batch, dim3((unsigned)total_fixed_blocks), dim3(256), 0, st, F, fixed_prefix, n,
                       (int)FX_ZERO);
    const Gpd32Args* T = (const Gpd32Args*)args_table;
    if (shape_order == 2)
        hipLaunchKernelGGL((k_gpd32_batch<2, TileCT<2, 4, 4, 4, false>>), dim3((unsigned)total_tiles), dim3(GPD32_BS), lds,
                           st, T, tile_prefix, n);
    else
        hipLaunchKernelGGL((k_gpd32_batch<3, TileCT<3, 4, 4, 4, false>>), dim3((unsigned)total_tiles), dim3(GPD32_BS), lds,
                           st, T, tile_prefix, n);
    hipLaunchKernelGGL(k_fixed_batch, dim3((unsigned)total_fixed_blocks), dim3(256), 0, st, F, fixed_prefix, n,
                       (int)FX_TO_F64);
    return hipGetLastError();
}

}  // namespace pp
