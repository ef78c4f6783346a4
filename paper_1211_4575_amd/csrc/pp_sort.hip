// Per-cell particle sort (Sec. III: between the particle and field updates the particle
// arrays are sorted by cell for cache locality).  Counting sort by tile-major cell key:
// histogram (atomics) -> exclusive scan -> scatter into the alternate buffers (atomic
// cursors, so the order inside a cell is unspecified) -> the buffers swap roles.  The
// scanned bin starts stay with the species: the tiled particle kernel reads each tile's
// range from them.
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
    int32_t* cursor;
    int split;  // 1: key from the cell index; 0: key from the FP64 position
};

template <typename T>
__global__ void __launch_bounds__(256) k_scatter(ScatterArgs<T> A) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.n) return;
    int32_t key;
    int32_t c = 0;
    if (A.split) {
        c = A.cell[p];
        key = key_cell(A.G, c);
    } else {
        key = key_f64(A.G, (double)A.pos[0][p], (double)A.pos[1][p], (double)A.pos[2][p]);
    }
    const int32_t dst = atomicAdd(A.cursor + key, 1);
    if (A.split) A.cell_o[dst] = c;
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

template <typename T>
static hipError_t sort_species(pp_run* r, int s) {
    Species& S = r->sp[s];
    const KeyGeom G = key_geom(r);
    const int64_t nbins = r->g.nbins;
    const bool split = r->p.precision == PP_PREC_FP32_SPLIT;
    int32_t* off = S.offsets;
    const int bs = 256;
    const unsigned fill_grid = (unsigned)((nbins + 1 + bs - 1) / bs < 65535 ? (nbins + 1 + bs - 1) / bs : 65535);
    hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid), dim3(bs), 0, r->stream, off, nbins + 1, 0);
    if (S.n > 0) {
        const unsigned pg = (unsigned)((S.n + bs - 1) / bs);
        if (split)
            hipLaunchKernelGGL(k_hist_cell, dim3(pg), dim3(bs), 0, r->stream, G, (const int32_t*)S.cur.cell, S.n, off);
        else
            hipLaunchKernelGGL(k_hist_f64, dim3(pg), dim3(bs), 0, r->stream, G, (const double*)S.cur.pos[0],
                               (const double*)S.cur.pos[1], (const double*)S.cur.pos[2], S.n, off);
    }
    scan_inplace(off, nbins + 1, r->scan_tmp, r->stream);
    if (S.n > 0) {
        hipLaunchKernelGGL(k_copy_i32, dim3(fill_grid), dim3(bs), 0, r->stream, r->sort_cursor, (const int32_t*)off,
                           nbins);
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
