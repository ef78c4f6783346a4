// Per-cell particle sort (Sec. III: between the particle and field updates the particle
// arrays are sorted by cell for cache locality).
//
// FP64 form: counting sort by tile-major cell key (histogram -> exclusive scan -> scatter
// with atomic cursors; order inside a cell unspecified).
//
// Split form: particles are laid out tile by tile (64 cells).  Every particle has a rank r
// inside its cell; a tile's particles are laid out in pairs of ranks (see pair_table below):
// pair round R holds, for every cell with at least 2R + 2 particles, its particles of ranks
// 2R and 2R + 1, and the pairs, numbered round by round with cells ascending, come in chunks
// of 64 -- 128 slots, the first particles of the chunk's pairs, then their second particles
// in the same order -- so that a wavefront taking 128 slots holds in lanes l and 64 + l two
// particles of one cell, and in a full round its 64 lanes hold the tile's 64 cells in order.
// The pairs past the last whole chunk and the last particle of a cell with an odd count
// follow singly, rank by rank, cells ascending; ranks of SORT_RCAP and beyond come last.
// After a push the particle kernel has already counted the particles of every new cell and
// ranked each particle inside it, so the sort is a per-tile round table, a scan over tiles
// and the destination slot of every particle, kept as a permutation (ranked sort): the next
// particle kernel moves the particles while it updates them, and reading them (or any other
// use of the order) applies the permutation first; batched runs do the same, with every
// phase one launch over all members.  The first sort of a
// species (arbitrary order) buckets by tile -- a count per tile, a scan, and a scatter whose
// positions come from block-aggregated atomics -- and then rebuilds the tile order tile by
// tile.
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

// Block-level aggregation for the bucketing sort: a block of 256 threads handles 1024
// consecutive particles; each wavefront groups its lanes by destination tile (ballot loop),
// the group leader reserves slots in a small LDS table keyed by tile, and after a barrier
// one global atomic per distinct tile of the block reserves the block's run in that tile.
// When a block's particles come from one or two source tiles, its destinations are a few
// tiles of their neighbourhood; in arbitrary order (a fresh load) nearly every particle of a
// block has its own tile, the table fills at once and the probe limit sends the rest straight
// to the global counters.
constexpr int AGG_SLOTS = 128;
constexpr int AGG_PROBES = 8;
constexpr int AGG_PER_THREAD = 4;
constexpr int AGG_BLOCK = 256 * AGG_PER_THREAD;

// LDS slot of a key (open addressing, at most AGG_PROBES probes); -1 when none is free
__device__ __forceinline__ int agg_slot(int32_t* keys, int32_t key) {
    const unsigned h = ((unsigned)key * 2654435761u) >> 25;  // 7 bits
    for (int probe = 0; probe < AGG_PROBES; ++probe) {
        const int sl = (int)((h + (unsigned)probe) & (AGG_SLOTS - 1));
        const int32_t prev = atomicCAS(&keys[sl], -1, key);
        if (prev == -1 || prev == key) return sl;
    }
    return -1;
}

__device__ __forceinline__ void tile_count_block(const KeyGeom& G, const int32_t* __restrict__ cell, int64_t n,
                                                 int32_t* __restrict__ count, int64_t blk) {
    __shared__ int32_t keys[AGG_SLOTS];
    __shared__ int32_t cnt[AGG_SLOTS];
    for (int i = threadIdx.x; i < AGG_SLOTS; i += 256) {
        keys[i] = -1;
        cnt[i] = 0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t base = blk * AGG_BLOCK;
    for (int k = 0; k < AGG_PER_THREAD; ++k) {
        const int64_t p = base + k * 256 + threadIdx.x;
        const bool active = p < n;
        const int32_t tile = active ? key_cell(G, cell[p]) / TILE_CELLS : 0;
        uint64_t todo = __ballot(active);
        while (todo) {
            const int leader = __ffsll((unsigned long long)todo) - 1;
            const int32_t lk = __shfl(tile, leader, 64);
            const uint64_t grp = __ballot(active && tile == lk) & todo;
            if (lane == leader) {
                const int sl = agg_slot(keys, lk);
                if (sl >= 0)
                    atomicAdd(&cnt[sl], (int32_t)__popcll(grp));
                else
                    atomicAdd(count + lk, (int32_t)__popcll(grp));
            }
            todo &= ~grp;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < AGG_SLOTS; i += 256)
        if (keys[i] >= 0 && cnt[i] > 0) atomicAdd(count + keys[i], cnt[i]);
}

__global__ void __launch_bounds__(256) k_tile_count(KeyGeom G, const int32_t* __restrict__ cell, int64_t n,
                                                    int32_t* __restrict__ count) {
    tile_count_block(G, cell, n, count, blockIdx.x);
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
    int32_t* cursor;  // FP64 form: cell-bin starts (consumed); split form: tile starts (consumed)
};

template <typename T>
__global__ void __launch_bounds__(256) k_scatter(ScatterArgs<T> A) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.n) return;
    const int32_t key = key_f64(A.G, (double)A.pos[0][p], (double)A.pos[1][p], (double)A.pos[2][p]);
    const int32_t dst = atomicAdd(A.cursor + key, 1);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        A.pos_o[d][dst] = A.pos[d][p];
        A.u_o[d][dst] = A.u[d][p];
    }
    if (A.id) A.id_o[dst] = A.id[p];
}

// split form: bucket by tile with block-level aggregation (see k_tile_count); a wavefront's
// particles bound for one tile get consecutive slots in their source order
template <typename T>
__device__ __forceinline__ void scatter_tiles_block(const ScatterArgs<T>& A, int64_t blk) {
    __shared__ int32_t keys[AGG_SLOTS];
    __shared__ int32_t cnt[AGG_SLOTS];
    __shared__ int32_t gbase[AGG_SLOTS];
    for (int i = threadIdx.x; i < AGG_SLOTS; i += 256) {
        keys[i] = -1;
        cnt[i] = 0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t base = blk * AGG_BLOCK;
    int my_slot[AGG_PER_THREAD];
    int32_t my_off[AGG_PER_THREAD];
#pragma unroll
    for (int k = 0; k < AGG_PER_THREAD; ++k) {
        const int64_t p = base + k * 256 + threadIdx.x;
        const bool active = p < A.n;
        const int32_t tile = active ? key_cell(A.G, A.cell[p]) / TILE_CELLS : 0;
        my_slot[k] = -2;
        my_off[k] = 0;
        uint64_t todo = __ballot(active);
        while (todo) {
            const int leader = __ffsll((unsigned long long)todo) - 1;
            const int32_t lk = __shfl(tile, leader, 64);
            const uint64_t grp = __ballot(active && tile == lk) & todo;
            int sl = 0;
            int32_t off = 0;
            if (lane == leader) {
                sl = agg_slot(keys, lk);
                if (sl >= 0)
                    off = atomicAdd(&cnt[sl], (int32_t)__popcll(grp));
                else
                    off = atomicAdd(A.cursor + lk, (int32_t)__popcll(grp));  // table full: direct
            }
            sl = __shfl(sl, leader, 64);
            off = __shfl(off, leader, 64);
            if ((grp >> lane) & 1ull) {
                my_slot[k] = sl;
                my_off[k] = off + (int32_t)__popcll(grp & ((1ull << lane) - 1ull));
            }
            todo &= ~grp;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < AGG_SLOTS; i += 256)
        if (keys[i] >= 0) gbase[i] = atomicAdd(A.cursor + keys[i], cnt[i]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < AGG_PER_THREAD; ++k) {
        const int64_t p = base + k * 256 + threadIdx.x;
        if (p >= A.n || my_slot[k] == -2) continue;
        const int32_t dst = my_slot[k] >= 0 ? gbase[my_slot[k]] + my_off[k] : my_off[k];
        A.cell_o[dst] = A.cell[p];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            A.pos_o[d][dst] = A.pos[d][p];
            A.u_o[d][dst] = A.u[d][p];
        }
        if (A.id) A.id_o[dst] = A.id[p];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_scatter_tiles(ScatterArgs<T> A) {
    scatter_tiles_block(A, blockIdx.x);
}

// largest tile population (the fixed-point current's scale depends on it)
__global__ void __launch_bounds__(256) k_tile_max(const int32_t* __restrict__ start, int64_t ntiles, int32_t* out) {
    int m = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += (int64_t)gridDim.x * blockDim.x) {
        const int c = start[t + 1] - start[t];
        m = c > m ? c : m;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int other = __shfl_xor(m, o, 64);
        m = other > m ? other : m;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

// The round table of one tile, built by one wavefront with lane = local cell, k = the
// particles the lane's cell holds in the table (min(count, SORT_RCAP)), rmax = the largest k:
// entry r (r < rmax) goes to put(r, entry), called by lane r - base in the pass over ranks
// base .. base + 63.  nchunk = whole chunks of 64 pairs, intable = particles in the table.
template <class Put>
__device__ __forceinline__ void pair_table(int k, int rmax, Put put, int32_t& nchunk, int32_t& intable) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = lane == 0 ? 0ull : ((1ull << lane) - 1ull);
    int pairs = k >> 1;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) pairs += __shfl_xor(pairs, o, 64);
    nchunk = pairs >> 6;
    int32_t pb = 0, sb = 0;  // pairs of the rounds before, single particles of the ranks before
    for (int base = 0; base < rmax; base += 64) {
        const int nr = rmax - base < 64 ? rmax - base : 64;
        RoundEntry mine{0ull, 0ull, 0, 0};
        // the two ranks 2R, 2R + 1 of a pair round share its pair mask (base is even)
        for (int rr = 0; rr < nr; rr += 2) {
            const int r = base + rr;
            const uint64_t pm = __ballot(k >= r + 2);  // cells with a pair of ranks r, r + 1
            const int32_t g = pb + (int32_t)__popcll(pm & below);
            const bool chunked = ((pm >> lane) & 1ull) && g < (nchunk << 6);
            const uint64_t sm0 = __ballot(k > r && !chunked);
            const uint64_t sm1 = __ballot(k > r + 1 && !chunked);
            const int32_t sb1 = sb + (int32_t)__popcll(sm0);
            if (lane == rr || lane == rr + 1) {
                mine.pmask = pm;
                mine.smask = lane == rr ? sm0 : sm1;
                mine.pbefore = pb;
                mine.sbefore = lane == rr ? sb : sb1;
            }
            // a last rank without its partner (nr odd) counts only its own single particles
            sb = rr + 1 < nr ? sb1 + (int32_t)__popcll(sm1) : sb1;
            pb += (int32_t)__popcll(pm);
        }
        if (lane < nr) put(base + lane, mine);
    }
    intable = (nchunk << 7) + sb;
}

// Slot inside its tile of the rank-r particle (r < SORT_RCAP) of local cell lc.
__device__ __forceinline__ int32_t pair_slot(const RoundEntry& e, int32_t nchunk, int r, int lc) {
    const uint64_t below = lc == 0 ? 0ull : ((1ull << lc) - 1ull);
    if ((e.pmask >> lc) & 1ull) {
        const int32_t g = e.pbefore + (int32_t)__popcll(e.pmask & below);
        if (g < (nchunk << 6)) return ((g >> 6) << 7) + ((r & 1) << 6) + (g & 63);
    }
    return (nchunk << 7) + e.sbefore + (int32_t)__popcll(e.smask & below);
}

// Rebuild of one tile in the tile order (one workgroup per tile): ranks inside cells from LDS
// atomics, the round table from ballots over the 64 cells, then a gather copy so the
// writes are coalesced (the reads stay inside the tile's segment).
constexpr int REORDER_RMAX = 1024;

template <typename T>
struct ReorderArgs {
    KeyGeom G;
    int64_t ntiles;
    const int32_t* start;
    const int32_t* cell;
    const T* pos[3];
    const T* u[3];
    const int64_t* id;
    int32_t* cell_o;
    T* pos_o[3];
    T* u_o[3];
    int64_t* id_o;
    int32_t* rank;  // scratch, one per particle
    int32_t* perm;  // scratch, one per particle
};

template <typename T>
__device__ __forceinline__ void tile_reorder_tile(const ReorderArgs<T>& A, int64_t tile) {
    __shared__ int32_t cnt[TILE_CELLS];
    __shared__ RoundEntry tab[SORT_RCAP];
    __shared__ int32_t nch, intab;
    __shared__ int32_t ovf;
    if (tile >= A.ntiles) return;
    const int32_t s = A.start[tile], e = A.start[tile + 1];
    if (threadIdx.x < TILE_CELLS) cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) ovf = 0;
    __syncthreads();
    for (int32_t i = s + threadIdx.x; i < e; i += 256) {
        const int32_t lc = key_cell(A.G, A.cell[i]) % TILE_CELLS;
        int32_t r = atomicAdd(&cnt[lc], 1);
        r = r < REORDER_RMAX ? r : REORDER_RMAX;
        A.rank[i] = (lc << 24) | r;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int k = cnt[lane] < SORT_RCAP ? cnt[lane] : SORT_RCAP;
        int mx = k;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int other = __shfl_xor(mx, o, 64);
            mx = other > mx ? other : mx;
        }
        int32_t nc, it;
        pair_table(k, mx, [&](int r, const RoundEntry& en) { tab[r] = en; }, nc, it);
        if (lane == 0) {
            nch = nc;
            intab = it;
        }
    }
    __syncthreads();
    for (int32_t i = s + threadIdx.x; i < e; i += 256) {
        const int32_t rk = A.rank[i];
        const int lc = rk >> 24;
        const int r = rk & 0xFFFFFF;
        const int32_t pos = r < SORT_RCAP ? pair_slot(tab[r], nch, r, lc) : intab + atomicAdd(&ovf, 1);
        A.perm[s + pos] = i;
    }
    __threadfence_block();
    __syncthreads();
    for (int32_t j = s + threadIdx.x; j < e; j += 256) {
        const int32_t i = A.perm[j];
        A.cell_o[j] = A.cell[i];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            A.pos_o[d][j] = A.pos[d][i];
            A.u_o[d][j] = A.u[d][i];
        }
        if (A.id) A.id_o[j] = A.id[i];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_tile_reorder(ReorderArgs<T> A) {
    tile_reorder_tile(A, blockIdx.x);
}

// ---- ranked sort (split form, after a push) ---------------------------------------------
// The particle kernel left, for species s, the number of particles of each cell at the new
// positions (cnt) and each particle's rank among the particles of its new cell.  Round r of
// a tile holds the rank-r particle of every cell with more than r particles, in cell order,
// so the particle of rank r in local cell lc goes to
//   tile start + sum over cells of min(count, r) + #{cells c < lc with count > r};
// the first two terms come from a per-tile round table.  Ranks of SORT_RCAP and beyond go
// to an overflow tail of the tile (order there unspecified).

struct RankedArgs {
    KeyGeom G;
    int64_t ntiles;
    int32_t* cnt;           // per cell (read and cleared by the table kernel)
    RoundEntry* rounds;     // ntiles * SORT_RCAP
    int32_t* tot;           // ntiles + 1: tile totals, scanned into the next tile starts
    int32_t* rtot;          // ntiles: particles in the table's rounds
    int32_t* nchunk;        // ntiles: whole chunks of 64 pairs
    int32_t* ovf;           // ntiles: overflow cursors
    int32_t* tile_max;      // largest tile population
    const int32_t* start;   // current tile starts (source order)
    const int32_t* rank;
    int64_t n;
    const int32_t* cell;
    const float* pos[3];
    const float* u[3];
    const int64_t* id;
    int32_t* cell_o;
    float* pos_o[3];
    float* u_o[3];
    int64_t* id_o;
};

// one wavefront per tile: lane = local cell
__device__ __forceinline__ void round_table_tile(const RankedArgs& A, int64_t t) {
    const int lane = threadIdx.x & 63;
    if (t >= A.ntiles) return;
    const KeyGeom& G = A.G;
    const int ti = (int)(t % G.nt[0]), tj = (int)((t / G.nt[0]) % G.nt[1]), tk = (int)(t / ((int64_t)G.nt[0] * G.nt[1]));
    const int li = lane % G.t[0], lj = (lane / G.t[0]) % G.t[1], lk = lane / (G.t[0] * G.t[1]);
    const int i = ti * G.t[0] + li, j = tj * G.t[1] + lj, k = tk * G.t[2] + lk;
    int c = 0;
    if (i < G.n[0] && j < G.n[1] && k < G.n[2]) {
        const int64_t g = (int64_t)i + (int64_t)G.n[0] * (j + (int64_t)G.n[1] * k);
        c = A.cnt[g];
        A.cnt[g] = 0;
    }
    int tot = c, mx = c;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        tot += __shfl_xor(tot, o, 64);
        const int other = __shfl_xor(mx, o, 64);
        mx = other > mx ? other : mx;
    }
    const int rmax = mx < SORT_RCAP ? mx : SORT_RCAP;
    const int kc = c < SORT_RCAP ? c : SORT_RCAP;
    int32_t nchunk, intable;
    pair_table(kc, rmax, [&](int r, const RoundEntry& e) { A.rounds[t * SORT_RCAP + r] = e; }, nchunk, intable);
    if (lane == 0) {
        A.tot[t] = tot;
        A.rtot[t] = intable;
        A.nchunk[t] = nchunk;
        A.ovf[t] = 0;
        // one address for every tile: read first (the value only grows, so a stale read
        // can only cause an unneeded atomic), so that few of the atomics are issued
        if (tot > *(volatile int32_t*)A.tile_max) atomicMax(A.tile_max, tot);
        if (t == A.ntiles - 1) A.tot[A.ntiles] = 0;
    }
}

__global__ void __launch_bounds__(256) k_round_tables(RankedArgs A) {
    round_table_tile(A, (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
}

// Destination slots of PERM_PER particles per thread, p = p0 + 256 k below pend: the table
// position of rank r in the new cell's tile (tot holds the next tile starts), or -1 for a
// flagged particle (negative rank) and for inconsistent counts (flagged state: never past the
// tile).  Every load of every particle is issued before any result is used, so the
// dependent loads of several particles are in flight together.  Ranks past the round table
// take slots at the end of their tile with one atomic per wavefront and tile, lanes in lane
// order (bunched plasmas put hundreds of particles in one cell).  Called by whole wavefronts.
constexpr int PERM_PER = 4;
constexpr int PERM_BLOCK = 256 * PERM_PER;

__device__ __forceinline__ void ranked_slots(const RankedArgs& A, int64_t p0, int64_t pend, int32_t pos[PERM_PER]) {
    int32_t r[PERM_PER], c[PERM_PER], t[PERM_PER], lim[PERM_PER];
#pragma unroll
    for (int k = 0; k < PERM_PER; ++k) {
        const int64_t p = p0 + k * 256;
        const bool v = p < pend;
        r[k] = v ? A.rank[p] : -1;
        c[k] = v ? A.cell[p] : 0;
    }
    // the table reads of every particle, issued together and unconditionally (a particle
    // without a slot reads its tile's first entries and ignores them), then the slots
    int32_t lc[PERM_PER], base[PERM_PER], nch[PERM_PER], rt[PERM_PER];
    RoundEntry e[PERM_PER];
#pragma unroll
    for (int k = 0; k < PERM_PER; ++k) {
        const int32_t key = key_cell(A.G, r[k] < 0 ? 0 : c[k]);
        t[k] = key / TILE_CELLS;
        lc[k] = key % TILE_CELLS;
    }
#pragma unroll
    for (int k = 0; k < PERM_PER; ++k) {
        base[k] = A.tot[t[k]];
        lim[k] = A.tot[t[k] + 1];
        nch[k] = A.nchunk[t[k]];
        rt[k] = A.rtot[t[k]];
        e[k] = A.rounds[(int64_t)t[k] * SORT_RCAP + (r[k] >= 0 && r[k] < SORT_RCAP ? r[k] : 0)];
    }
#pragma unroll
    for (int k = 0; k < PERM_PER; ++k) {
        // computed for every particle and selected (no branch the table reads could sink into)
        const bool in_table = r[k] >= 0 && r[k] < SORT_RCAP;
        const int32_t ps = pair_slot(e[k], nch[k], in_table ? r[k] : 0, lc[k]);
        pos[k] = r[k] < 0 ? -1 : base[k] + (in_table ? ps : rt[k]);
    }
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < PERM_PER; ++k) {
        const bool over = r[k] >= SORT_RCAP;
        uint64_t todo = __ballot(over);
        while (todo) {
            const int leader = __ffsll((unsigned long long)todo) - 1;
            const int32_t lt = __shfl(t[k], leader, 64);
            const uint64_t grp = __ballot(over && t[k] == lt) & todo;
            int32_t base = 0;
            if (lane == leader) base = atomicAdd(&A.ovf[lt], (int32_t)__popcll(grp));
            base = __shfl(base, leader, 64);
            if (over && t[k] == lt) pos[k] += base + (int32_t)__popcll(grp & ((1ull << lane) - 1ull));
            todo &= ~grp;
        }
    }
#pragma unroll
    for (int k = 0; k < PERM_PER; ++k)
        if (r[k] < 0 || pos[k] >= lim[k]) pos[k] = -1;
}

// perm[slot] = particle for the particles of source tile T (one workgroup per tile).  Most
// of them stay in the tile: their entries are collected in an LDS image of T's destination
// range and written out in order (entries that particles from neighbouring tiles fill are
// written by those tiles' workgroups, directly); the rest, and every entry of a destination
// range larger than the image, are written directly.
constexpr int PERM_IMG = 4096;

__device__ __forceinline__ void ranked_perm_tile(const RankedArgs& A, int32_t* perm, int64_t T, int32_t* img) {
    if (T >= A.ntiles) return;
    const int32_t ss = A.start[T], se = A.start[T + 1];
    const int32_t d0 = A.tot[T];
    const int32_t nd = A.tot[T + 1] - d0;
    const bool staged = nd <= PERM_IMG;
    if (staged)
        for (int32_t q = threadIdx.x; q < nd; q += blockDim.x) img[q] = -1;
    __syncthreads();
    for (int64_t b = ss; b < se; b += PERM_BLOCK) {
        int32_t pos[PERM_PER];
        ranked_slots(A, b + threadIdx.x, se, pos);
#pragma unroll
        for (int k = 0; k < PERM_PER; ++k) {
            if (pos[k] < 0) continue;
            const int32_t p = (int32_t)(b + threadIdx.x + k * 256);
            const int32_t q = pos[k] - d0;
            if (staged && q >= 0 && q < nd)
                img[q] = p;
            else
                perm[pos[k]] = p;
        }
    }
    __syncthreads();
    if (staged)
        for (int32_t q = threadIdx.x; q < nd; q += blockDim.x) {
            const int32_t v = img[q];
            if (v >= 0) perm[d0 + q] = v;
        }
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


static unsigned grid_for(int64_t n, int bs, int64_t cap = 65535) {
    int64_t g = (n + bs - 1) / bs;
    if (g > cap) g = cap;
    return (unsigned)(g < 1 ? 1 : g);
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

// ---- batched ranked sort of one species slot over several runs -----------------------------
struct SortDesc {
    RankedArgs A;
    int32_t* perm;  // n slots: the destination order, perm[slot] = particle
};

// reset: tile maximum and perm = -1; tables: round tables; scan: next tile starts;
// perm: every particle's slot
enum SortPhase { SP_RESET = 0, SP_TABLES = 1, SP_SCAN = 2, SP_PERM = 3 };

// whole-segment exclusive scan by one workgroup (segments are short: one entry per tile)
__device__ __forceinline__ void scan_segment(int32_t* data, int64_t n) {
    __shared__ int32_t sh[256];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < n; base += 256) {
        const int64_t q = base + threadIdx.x;
        const int32_t v = q < n ? data[q] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int32_t x = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += x;
            __syncthreads();
        }
        const int32_t incl = sh[threadIdx.x];
        if (q < n) data[q] = carry + incl - v;
        __syncthreads();
        if (threadIdx.x == 255) carry += incl;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_sort_batch(const SortDesc* __restrict__ T, const int64_t* __restrict__ prefix,
                                                    int nseg, int phase) {
    const int64_t b = blockIdx.x;
    const int r = find_segment(prefix, nseg, b);
    if (r < 0) return;
    const RankedArgs& A = T[r].A;
    const int64_t blk = b - prefix[r];
    const int64_t p = blk * 256 + threadIdx.x;
    switch (phase) {
    case SP_RESET:
        if (p == 0) *A.tile_max = 0;
        if (p < A.n) T[r].perm[p] = -1;
        break;
    case SP_TABLES:
        round_table_tile(A, blk * 4 + (threadIdx.x >> 6));
        break;
    case SP_SCAN:
        scan_segment(A.tot, A.ntiles + 1);
        break;
    case SP_PERM: {
        __shared__ int32_t img[PERM_IMG];
        ranked_perm_tile(A, T[r].perm, blk, img);
        break;
    }
    default:
        break;
    }
}

static void ranked_args(const pp_run* r, int s, RankedArgs* A) {
    const Species& S = r->sp[s];
    const int64_t nt = r->g.ntiles;
    A->G = key_geom(r);
    A->ntiles = nt;
    A->cnt = S.cell_cnt;
    A->rounds = r->rounds;
    A->tot = S.offsets_next;
    A->rtot = r->sort_cursor;
    A->ovf = r->sort_cursor + nt;
    A->nchunk = r->sort_cursor + 2 * nt;
    A->tile_max = r->tile_max + s;
    A->start = S.offsets;
    A->rank = S.rank;
    A->n = S.n;
    A->cell = S.cur.cell;
    A->id = S.cur.id;
    A->cell_o = S.cur.cell_alt;
    A->id_o = S.cur.id ? S.cur.id_alt : nullptr;
    for (int d = 0; d < 3; ++d) {
        A->pos[d] = (const float*)S.cur.pos[d];
        A->u[d] = (const float*)S.cur.u[d];
        A->pos_o[d] = (float*)S.cur.pos_alt[d];
        A->u_o[d] = (float*)S.cur.u_alt[d];
    }
}

void sort_desc(const pp_run* r, int s, SortDesc* D) {
    ranked_args(r, s, &D->A);
    D->perm = r->sp[s].perm;
}

size_t sort_desc_size() { return sizeof(SortDesc); }

// Blocks each phase needs for one descriptor.
void sort_desc_blocks(const pp_run* r, int s, int64_t blocks[SORT_BATCH_PHASES]) {
    const int64_t nt = r->g.ntiles;
    const int64_t pb = (r->sp[s].n + 255) / 256;
    blocks[SP_RESET] = pb > 0 ? pb : 1;
    blocks[SP_TABLES] = (nt + 3) / 4;
    blocks[SP_SCAN] = 1;
    blocks[SP_PERM] = r->sp[s].n > 0 ? nt : 0;
}

// prefixes: one array of nseg + 1 block prefixes (device) per phase, totals: blocks per phase
hipError_t launch_sort_batch(const void* table, const int64_t* const prefixes[SORT_BATCH_PHASES],
                             const int64_t totals[SORT_BATCH_PHASES], int nseg, hipStream_t st) {
    if (nseg == 0) return hipSuccess;
    const SortDesc* T = (const SortDesc*)table;
    for (int ph = 0; ph < SORT_BATCH_PHASES; ++ph) {
        if (totals[ph] == 0) continue;
        hipLaunchKernelGGL(k_sort_batch, dim3((unsigned)totals[ph]), dim3(256), 0, st, T, prefixes[ph], nseg, ph);
    }
    return hipGetLastError();
}

void swap_buffers(pp_particles& c) {
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

// Host bookkeeping once a ranked sort is enqueued: the new tile starts become current and the
// particles stay where they are until the next particle kernel (or materialize) moves them.
void sort_enqueued(pp_run* r, int s) {
    Species& S = r->sp[s];
    int32_t* t = S.offsets;
    S.offsets = S.offsets_next;
    S.offsets_next = t;
    S.ranked = false;
    S.sorted = true;
    S.pending = S.n > 0;
}

// Destination slot of every particle, as a permutation: perm[slot] = particle (slots no
// particle goes to keep -1).  The particle kernel then reads through it and writes the
// new order, so the particles move once per step, together with their update.
__global__ void __launch_bounds__(256) k_ranked_perm(RankedArgs A, int32_t* perm) {
    __shared__ int32_t img[PERM_IMG];
    ranked_perm_tile(A, perm, blockIdx.x, img);
}

// out[q] = in[perm[q]] for every attribute (the move a pending permutation stands for)
struct ApplyArgs {
    int64_t n;
    const int32_t* perm;
    const int32_t* cell;
    const float* pos[3];
    const float* u[3];
    const int64_t* id;
    int32_t* cell_o;
    float* pos_o[3];
    float* u_o[3];
    int64_t* id_o;
};

__global__ void __launch_bounds__(256) k_apply_perm(ApplyArgs A) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= A.n) return;
    const int32_t p = A.perm[q];
    if (p < 0) return;
    A.cell_o[q] = A.cell[p];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        A.pos_o[d][q] = A.pos[d][p];
        A.u_o[d][q] = A.u[d][p];
    }
    if (A.id) A.id_o[q] = A.id[p];
}

hipError_t materialize(pp_run* r, int s) {
    for (int k = 0; k < PP_MAX_SPECIES; ++k) {
        if (s >= 0 && k != s) continue;
        Species& S = r->sp[k];
        if (!S.active || !S.pending) continue;
        if (S.n > 0) {
            ApplyArgs A;
            A.n = S.n;
            A.perm = S.perm;
            A.cell = S.cur.cell;
            A.cell_o = S.cur.cell_alt;
            A.id = S.cur.id;
            A.id_o = S.cur.id ? S.cur.id_alt : nullptr;
            for (int d = 0; d < 3; ++d) {
                A.pos[d] = (const float*)S.cur.pos[d];
                A.u[d] = (const float*)S.cur.u[d];
                A.pos_o[d] = (float*)S.cur.pos_alt[d];
                A.u_o[d] = (float*)S.cur.u_alt[d];
            }
            hipLaunchKernelGGL(k_apply_perm, dim3((unsigned)((S.n + 255) / 256)), dim3(256), 0, r->stream, A);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            swap_buffers(S.cur);
        }
        S.pending = false;
    }
    return hipSuccess;
}

static hipError_t sort_ranked(pp_run* r, int s) {
    RankedArgs A;
    ranked_args(r, s, &A);
    Species& S = r->sp[s];
    const int64_t nt = r->g.ntiles;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, r->stream, r->tile_max + s, (int64_t)1, 0);
    hipLaunchKernelGGL(k_round_tables, dim3((unsigned)((nt + 3) / 4)), dim3(256), 0, r->stream, A);
    scan_inplace(A.tot, nt + 1, r->scan_tmp, r->stream);
    if (S.n > 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(S.n, 256)), dim3(256), 0, r->stream, S.perm, S.n, -1);
        hipLaunchKernelGGL(k_ranked_perm, dim3((unsigned)nt), dim3(256), 0, r->stream, A, S.perm);
    }
    hipError_t e = hipGetLastError();
    sort_enqueued(r, s);
    return e;
}

template <typename T>
static hipError_t sort_species(pp_run* r, int s) {
    Species& S = r->sp[s];
    const KeyGeom G = key_geom(r);
    const int64_t nbins = r->g.nbins;
    const int64_t ntiles = r->g.ntiles;
    const bool split = r->p.precision == PP_PREC_FP32_SPLIT;
    const int bs = 256;
    const int64_t nkeys = split ? ntiles : nbins;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nkeys + 1, bs)), dim3(bs), 0, r->stream, S.offsets, nkeys + 1, 0);
    if (S.n > 0) {
        const unsigned pg = (unsigned)((S.n + bs - 1) / bs);
        if (split)
            hipLaunchKernelGGL(k_tile_count, dim3((unsigned)((S.n + AGG_BLOCK - 1) / AGG_BLOCK)), dim3(256), 0,
                               r->stream, G, (const int32_t*)S.cur.cell, S.n, S.offsets);
        else
            hipLaunchKernelGGL(k_hist_f64, dim3(pg), dim3(bs), 0, r->stream, G, (const double*)S.cur.pos[0],
                               (const double*)S.cur.pos[1], (const double*)S.cur.pos[2], S.n, S.offsets);
    }
    scan_inplace(S.offsets, nkeys + 1, r->scan_tmp, r->stream);
    if (split) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, r->stream, r->tile_max + s, (int64_t)1, 0);
        hipLaunchKernelGGL(k_tile_max, dim3(grid_for(ntiles, bs, 1024)), dim3(bs), 0, r->stream,
                           (const int32_t*)S.offsets, ntiles, r->tile_max + s);
    }
    if (S.n > 0) {
        hipLaunchKernelGGL(k_copy_i32, dim3(grid_for(nkeys, bs)), dim3(bs), 0, r->stream, r->sort_cursor,
                           (const int32_t*)S.offsets, nkeys);
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
        if (split)
            hipLaunchKernelGGL(k_scatter_tiles<T>, dim3((unsigned)((S.n + AGG_BLOCK - 1) / AGG_BLOCK)), dim3(256), 0,
                               r->stream, A);
        else
            hipLaunchKernelGGL(k_scatter<T>, dim3((unsigned)((S.n + bs - 1) / bs)), dim3(bs), 0, r->stream, A);
        swap_buffers(S.cur);
        if (split) {
            ReorderArgs<T> B;
            B.G = G;
            B.ntiles = ntiles;
            B.start = S.offsets;
            B.cell = S.cur.cell;
            B.id = S.cur.id;
            B.cell_o = S.cur.cell_alt;
            B.id_o = S.cur.id ? S.cur.id_alt : nullptr;
            for (int d = 0; d < 3; ++d) {
                B.pos[d] = (const T*)S.cur.pos[d];
                B.u[d] = (const T*)S.cur.u[d];
                B.pos_o[d] = (T*)S.cur.pos_alt[d];
                B.u_o[d] = (T*)S.cur.u_alt[d];
            }
            B.rank = r->sort_scratch;
            B.perm = r->sort_scratch + r->sort_scratch_n;
            hipLaunchKernelGGL(k_tile_reorder<T>, dim3((unsigned)ntiles), dim3(256), 0, r->stream, B);
            swap_buffers(S.cur);
        }
    }
    S.sorted = true;
    S.ranked = false;
    return hipGetLastError();
}

hipError_t launch_sort(pp_run* r, int s) {
    if (r->p.precision == PP_PREC_FP32_SPLIT) {
        hipError_t e = materialize(r, s);  // a sort of a sort: apply the pending order first
        if (e != hipSuccess) return e;
        return r->sp[s].ranked ? sort_ranked(r, s) : sort_species<float>(r, s);
    }
    return sort_species<double>(r, s);
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace pp
