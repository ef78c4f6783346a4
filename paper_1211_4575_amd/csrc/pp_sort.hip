// Per-cell particle sort (Sec. III: between the particle and field updates the particle
// arrays are sorted by cell for cache locality).
//
// FP64 form: counting sort by tile-major cell key (histogram -> exclusive scan -> scatter
// with atomic cursors; order inside a cell unspecified).
//
// Split form: "round-major" order inside each tile of 64 cells.  Every particle gets a
// rank r inside its cell; the tile's particles are laid out round by round (all rank-0
// particles of the tile's cells, then all rank-1 particles, ...), cells ascending inside a
// round.  A wavefront reading 64 consecutive particles therefore reads coalesced memory and
// its lanes sit in (almost always) 64 different cells, which keeps the LDS current
// accumulation of the particle kernel free of same-address collisions; every wavefront
// also gets a full 64 particles whatever the cell occupancy is.
//   histogram per cell -> per tile (one wavefront): round starts T[r] and the bit mask of
//   cells taking part M[r] (ballot over the 64 cells), tile totals -> scan over tiles ->
//   scatter: r = atomic rank in the cell, position = tile start + T[r] + popcount(M[r]
//   below the cell).  Ranks at or beyond the table capacity go to a per-tile overflow
//   segment at the end of the tile.
#include "pp_device.hpp"
#include "pp_internal.hpp"

namespace pp {

struct KeyGeom {
    int n[3];
    int t[3];
    int nt[3];
};

__device__ __forceinline__ int32_t tile_key(const KeyGeom& G, int i, int j, int k) {
    const int ti = i / G.t[0], tj = j / G.t[1], tk = k / G.t[2];
    const int li = i - ti * G.t[0], lj = j - tj * G.t[1], lk = k - tk * G.t[2];
    const int tile = ti + G.nt[0] * (tj + G.nt[1] * tk);
    return tile * TILE_CELLS + li + G.t[0] * (lj + G.t[1] * lk);
}

// key of an FP64 particle: nearest cell centre
__device__ __forceinline__ int32_t key_f64(const KeyGeom& G, double x, double y, double z) {
    int c[3];
    const double X[3] = {x, y, z};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int v = (int)floor(X[d] + 0.5);
        if (v >= G.n[d]) v -= G.n[d];
        if (v < 0) v += G.n[d];
        // positions outside [0, n) (not produced by the push) are binned into cell 0,
        // keeping every bin index in range; the particle kernel checks positions itself
        if (v < 0 || v >= G.n[d]) v = 0;
        c[d] = v;
    }
    return tile_key(G, c[0], c[1], c[2]);
}

__device__ __forceinline__ int32_t key_cell(const KeyGeom& G, int32_t cell) {
    // an index outside the box (not produced by the push) is binned with cell 0; the
    // particle kernel flags it when it finds the particle outside its tile
    if (cell < 0 || cell >= G.n[0] * G.n[1] * G.n[2]) cell = 0;
    const int i = cell % G.n[0];
    const int r = cell / G.n[0];
    const int j = r % G.n[1];
    const int k = r / G.n[1];
    return tile_key(G, i, j, k);
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        p[q] = v;
}

__global__ void k_copy_i32(int32_t* dst, const int32_t* src, int64_t n) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        dst[q] = src[q];
}

__global__ void __launch_bounds__(256) k_hist_f64(KeyGeom G, const double* __restrict__ x, const double* __restrict__ y,
                                                  const double* __restrict__ z, int64_t n, int32_t* count) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    atomicAdd(count + key_f64(G, x[p], y[p], z[p]), 1);
}

__global__ void __launch_bounds__(256) k_hist_cell(KeyGeom G, const int32_t* __restrict__ cell, int64_t n,
                                                   int32_t* count) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    atomicAdd(count + key_cell(G, cell[p]), 1);
}

// One wavefront per tile: lane c holds the count of cell c of the tile.
__global__ void __launch_bounds__(64) k_tile_rounds(const int32_t* __restrict__ count, int64_t ntiles, int rcap,
                                                    int32_t* __restrict__ T, uint64_t* __restrict__ M,
                                                    int32_t* __restrict__ tile_total, int32_t* __restrict__ ovf) {
    const int64_t tile = blockIdx.x;
    if (tile >= ntiles) return;
    const int lane = threadIdx.x;
    const int cnt = count[tile * TILE_CELLS + lane];
    int tot = cnt, mx = cnt;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        tot += __shfl_xor(tot, o, 64);
        int other = __shfl_xor(mx, o, 64);
        mx = other > mx ? other : mx;
    }
    const int rmax = mx < rcap ? mx : rcap;
    int32_t* Tt = T + tile * (int64_t)(rcap + 1);
    uint64_t* Mt = M + tile * (int64_t)rcap;
    int run = 0;
    for (int r = 0; r < rmax; ++r) {
        const uint64_t m = __ballot(cnt > r);
        if (lane == 0) {
            Tt[r] = run;
            Mt[r] = m;
        }
        run += __popcll(m);
    }
    if (lane == 0) {
        Tt[rcap] = run;  // start of the overflow segment
        tile_total[tile] = tot;
        ovf[tile] = 0;
    }
}

template <typename T>
struct ScatterArgs {
    KeyGeom G;
    int64_t n;
    const int32_t* cell;
    const T* pos[3];
    const T* u[3];
    const int64_t* id;
    int32_t* cell_o;
    T* pos_o[3];
    T* u_o[3];
    int64_t* id_o;
    int32_t* cursor;        // FP64 form: bin starts (consumed); split form: per-cell rank cursors
    const int32_t* tstart;  // split form: tile starts
    const int32_t* rT;
    const uint64_t* rM;
    int32_t* ovf;
    int rcap;
    int split;  // 1: round-major order from the cell index; 0: cell order from the FP64 position
};

template <typename T>
__global__ void __launch_bounds__(256) k_scatter(ScatterArgs<T> A) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.n) return;
    int32_t dst;
    int32_t c = 0;
    if (A.split) {
        c = A.cell[p];
        const int32_t key = key_cell(A.G, c);
        const int32_t tile = key / TILE_CELLS;
        const int lc = key - tile * TILE_CELLS;
        const int32_t r = atomicAdd(A.cursor + key, 1);
        const int32_t base = A.tstart[tile];
        if (r < A.rcap) {
            const uint64_t m = A.rM[(int64_t)tile * A.rcap + r];
            const uint64_t below = lc == 0 ? 0ull : (m & ((1ull << lc) - 1ull));
            dst = base + A.rT[(int64_t)tile * (A.rcap + 1) + r] + __popcll(below);
        } else {
            dst = base + A.rT[(int64_t)tile * (A.rcap + 1) + A.rcap] + atomicAdd(A.ovf + tile, 1);
        }
        A.cell_o[dst] = c;
    } else {
        const int32_t key = key_f64(A.G, (double)A.pos[0][p], (double)A.pos[1][p], (double)A.pos[2][p]);
        dst = atomicAdd(A.cursor + key, 1);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        A.pos_o[d][dst] = A.pos[d][p];
        A.u_o[d][dst] = A.u[d][p];
    }
    if (A.id) A.id_o[dst] = A.id[p];
}

// ---- exclusive scan of int32, in place ------------------------------------------------
constexpr int SCAN_BS = 256, SCAN_PER = 8, SCAN_CHUNK = SCAN_BS * SCAN_PER;

__global__ void __launch_bounds__(SCAN_BS) k_scan_chunks(int32_t* data, int64_t n, int32_t* sums) {
    __shared__ int32_t sh[2][SCAN_BS];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
    int32_t v[SCAN_PER];
    int32_t tot = 0;
#pragma unroll
    for (int e = 0; e < SCAN_PER; ++e) {
        int64_t q = base + e;
        v[e] = q < n ? data[q] : 0;
        tot += v[e];
    }
    int cur = 0;
    sh[0][threadIdx.x] = tot;
    __syncthreads();
    for (int off = 1; off < SCAN_BS; off <<= 1) {
        int32_t x = sh[cur][threadIdx.x];
        if ((int)threadIdx.x >= off) x += sh[cur][threadIdx.x - off];
        sh[cur ^ 1][threadIdx.x] = x;
        cur ^= 1;
        __syncthreads();
    }
    int32_t incl = sh[cur][threadIdx.x];
    int32_t run = incl - tot;  // exclusive prefix of this thread
#pragma unroll
    for (int e = 0; e < SCAN_PER; ++e) {
        int64_t q = base + e;
        if (q < n) data[q] = run;
        run += v[e];
    }
    if (threadIdx.x == SCAN_BS - 1) sums[blockIdx.x] = incl;
}

__global__ void __launch_bounds__(SCAN_BS) k_scan_add(int32_t* data, int64_t n, const int32_t* sums) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK;
    const int32_t add = sums[blockIdx.x];
    for (int e = threadIdx.x; e < SCAN_CHUNK; e += SCAN_BS) {
        int64_t q = base + e;
        if (q < n) data[q] += add;
    }
}

int64_t scan_tmp_size(int64_t n) {
    int64_t tot = 0;
    while (n > 1) {
        n = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
        tot += n + 1;
    }
    return tot + 16;
}

static void scan_inplace(int32_t* data, int64_t n, int32_t* tmp, hipStream_t st) {
    const int64_t nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    hipLaunchKernelGGL(k_scan_chunks, dim3((unsigned)nb), dim3(SCAN_BS), 0, st, data, n, tmp);
    if (nb > 1) {
        scan_inplace(tmp, nb, tmp + nb + 1, st);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(SCAN_BS), 0, st, data, n, (const int32_t*)tmp);
    }
}

static KeyGeom key_geom(const pp_run* r) {
    KeyGeom G;
    for (int d = 0; d < 3; ++d) {
        G.n[d] = r->g.n[d];
        G.t[d] = r->g.t[d];
        G.nt[d] = r->g.nt[d];
    }
    return G;
}

static unsigned grid_for(int64_t n, int bs, int64_t cap = 65535) {
    int64_t g = (n + bs - 1) / bs;
    if (g > cap) g = cap;
    return (unsigned)(g < 1 ? 1 : g);
}

template <typename T>
static hipError_t sort_species(pp_run* r, int s) {
    Species& S = r->sp[s];
    const KeyGeom G = key_geom(r);
    const int64_t nbins = r->g.nbins;
    const int64_t ntiles = r->g.ntiles;
    const bool split = r->p.precision == PP_PREC_FP32_SPLIT;
    const int bs = 256;
    int32_t* count = split ? r->sort_count : S.offsets;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nbins + 1, bs)), dim3(bs), 0, r->stream, count, split ? nbins : nbins + 1, 0);
    if (S.n > 0) {
        const unsigned pg = (unsigned)((S.n + bs - 1) / bs);
        if (split)
            hipLaunchKernelGGL(k_hist_cell, dim3(pg), dim3(bs), 0, r->stream, G, (const int32_t*)S.cur.cell, S.n, count);
        else
            hipLaunchKernelGGL(k_hist_f64, dim3(pg), dim3(bs), 0, r->stream, G, (const double*)S.cur.pos[0],
                               (const double*)S.cur.pos[1], (const double*)S.cur.pos[2], S.n, count);
    }
    if (split) {
        // per-tile round tables and totals; then tile starts
        hipLaunchKernelGGL(k_tile_rounds, dim3((unsigned)ntiles), dim3(64), 0, r->stream, (const int32_t*)count, ntiles,
                           r->rcap, r->round_T, r->round_M, S.offsets, r->tile_ovf);
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, r->stream, S.offsets + ntiles, (int64_t)1, 0);
        scan_inplace(S.offsets, ntiles + 1, r->scan_tmp, r->stream);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nbins, bs)), dim3(bs), 0, r->stream, r->sort_cursor, nbins, 0);
    } else {
        scan_inplace(S.offsets, nbins + 1, r->scan_tmp, r->stream);
        if (S.n > 0)
            hipLaunchKernelGGL(k_copy_i32, dim3(grid_for(nbins, bs)), dim3(bs), 0, r->stream, r->sort_cursor,
                               (const int32_t*)S.offsets, nbins);
    }
    if (S.n > 0) {
        ScatterArgs<T> A;
        A.G = G;
        A.n = S.n;
        A.cell = S.cur.cell;
        A.id = S.cur.id;
        A.cell_o = S.cur.cell_alt;
        A.id_o = S.cur.id ? S.cur.id_alt : nullptr;
        for (int d = 0; d < 3; ++d) {
            A.pos[d] = (const T*)S.cur.pos[d];
            A.u[d] = (const T*)S.cur.u[d];
            A.pos_o[d] = (T*)S.cur.pos_alt[d];
            A.u_o[d] = (T*)S.cur.u_alt[d];
        }
        A.cursor = r->sort_cursor;
        A.tstart = S.offsets;
        A.rT = r->round_T;
        A.rM = r->round_M;
        A.ovf = r->tile_ovf;
        A.rcap = r->rcap;
        A.split = split ? 1 : 0;
        hipLaunchKernelGGL(k_scatter<T>, dim3((unsigned)((S.n + bs - 1) / bs)), dim3(bs), 0, r->stream, A);
        // swap roles of the two buffers
        pp_particles& c = S.cur;
        int32_t* tc = c.cell;
        c.cell = c.cell_alt;
        c.cell_alt = tc;
        int64_t* ti = c.id;
        c.id = c.id_alt;
        c.id_alt = ti;
        for (int d = 0; d < 3; ++d) {
            void* tp = c.pos[d];
            c.pos[d] = c.pos_alt[d];
            c.pos_alt[d] = tp;
            void* tu = c.u[d];
            c.u[d] = c.u_alt[d];
            c.u_alt[d] = tu;
        }
    }
    S.sorted = true;
    return hipGetLastError();
}

hipError_t launch_sort(pp_run* r, int s) {
    if (r->p.precision == PP_PREC_FP32_SPLIT) return sort_species<float>(r, s);
    return sort_species<double>(r, s);
}

}  // namespace pp
