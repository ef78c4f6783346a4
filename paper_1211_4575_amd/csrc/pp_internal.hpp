// Internal declarations of libpp (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/pp.h"

namespace pp {

// Tile-major cell keys: the box is cut into tiles of TILE_CELLS cells (tx*ty*tz = 64,
// one cell per lane of a wavefront); key = tile * 64 + local cell.  Tiles at the upper
// edge may be partial (cells outside the box never receive particles).
constexpr int TILE_CELLS = 64;
// LDS halo of the field tile (nodes below / above the tile) and of the current tile.  A split
// particle's offset lies in [lo, lo + 2) (lo = -1/2 for O = 2, 0 for O = 3), so its supports
// start between 2 nodes below and 1 node above its cell; the current window (O + 2 nodes
// per axis, covering the old and the new support) ends at most O + 1 nodes above its start.
constexpr int FLD_LO = 2;
constexpr int fld_hi(int O) { return O == 2 ? 2 : 3; }
constexpr int cur_lo(int) { return 2; }
constexpr int cur_hi(int O) { return O + 1; }

struct Geom {
    int n[3];       // cells
    int t[3];       // tile dims
    int nt[3];      // tiles per dim
    int64_t ncell;  // n0*n1*n2
    int64_t ntiles;
    int64_t nbins;  // ntiles * 64
};

struct Species {
    bool active = false;
    double q = 0, m = 1, w = 0;
    int64_t n = 0;
    pp_particles cur{};  // buffers read by the next push
    bool sorted = false;
    // FP64 form: nbins + 1 cell-bin starts.  Split form: ntiles + 1 tile starts of the
    // tile order of pp_sort.hip (valid when sorted).
    int32_t* offsets = nullptr;
    // split form, filled by the particle kernel for the next sort: particles per cell of the
    // new positions (ncell, zero between steps), each particle's rank among the particles of
    // its new cell (n; -1 for a particle found outside its tile), the next tile starts
    int32_t* cell_cnt = nullptr;
    int32_t* rank = nullptr;
    int32_t* offsets_next = nullptr;
    bool ranked = false;  // cell_cnt / rank describe the current positions
    // split form: the last sort left its order as a permutation (slot q of the new order is
    // particle perm[q] of the current buffers); the next particle kernel, or materialize,
    // moves the particles
    int32_t* perm = nullptr;
    bool pending = false;
};

// Round table of a tile (split-form sort), entry r for the particles of rank r in their cell
// (see pp_sort.hip for the order it encodes): pmask, the cells holding a pair of ranks
// 2R, 2R + 1 (R = r / 2), and pbefore, the pairs of rounds before R; smask, the cells whose
// rank-r particle is laid out singly, and sbefore, the single particles of ranks before r.
struct RoundEntry {
    uint64_t pmask;
    uint64_t smask;
    int32_t pbefore;
    int32_t sbefore;
};
constexpr int SORT_RCAP = 96;  // ranks per tile table (even); ranks beyond go to an overflow tail

// Line-solve stencil of one axis: out[i] = sum_j coef[j] * in[(i + off + j) mod n].
struct LineStencil {
    double* coef = nullptr;  // device
    int len = 0;
    int off = 0;
};

}  // namespace pp

struct pp_run {
    pp_params p{};
    pp_mesh mesh{};
    hipStream_t stream = nullptr;
    pp::Geom g{};
    pp::Species sp[PP_MAX_SPECIES];

    double* J2 = nullptr;      // second-order current (field order > 2)
    double* Bn = nullptr;      // copy of B^n during the field step
    double* Bw = nullptr;      // relaxation ping-pong partner
    double* R = nullptr;       // right-hand side of the elliptic equation
    double* rho = nullptr;     // charge density (diagnostics)
    double* rho_prev = nullptr;
    int64_t rho_prev_step = -1;
    int32_t* sort_cursor = nullptr;   // nbins: scatter cursors (cell bins or tiles)
    pp::RoundEntry* rounds = nullptr; // split form: ntiles * SORT_RCAP round tables
    int32_t* scan_tmp = nullptr;      // block sums of the scan
    int32_t* sort_scratch = nullptr;  // split form: rank and permutation of the tile-order rebuild
    int64_t sort_scratch_n = 0;       // particles per half of sort_scratch
    long long* Jq = nullptr;          // split form: current in 64-bit fixed point (3*ncell)
    int32_t* tile_max = nullptr;      // split form: largest particle count of a tile, per species
    double* qscale = nullptr;         // split form: 2^e of the fixed-point current (device)
    int32_t* flags = nullptr;        // device error flags
    double* dacc = nullptr;          // device accumulators for diagnostics
    pp::LineStencil line[3];

    // field-step constants
    double lap[3][16] = {};  // Laplacian stencil per axis, offsets -R..R (1/d^2 folded)
    int lap_r = 0;
    double diagA = 1.0;      // diagonal of (1 - alpha^2 c^2 dt^2 lap) on this grid
    double jac_rho = 0.0;    // spectral radius of the plain Jacobi iteration
    double relax_gamma = 1.0;  // Jacobi extrapolation factor
    double relax_r = 0.0;    // spectral radius of the extrapolated iteration
    int jac_sweeps = 0;      // relaxation sweeps per field step
    double jac_bound = 0.0;  // error reduction bound after jac_sweeps sweeps
    bool jac_converged = true;  // jac_bound <= relax_tol (false: capped by relax_max_iter)
    // the right-hand side of the last field step is still in R (for the measured residual),
    // with the alpha^2 c^2 dt^2 of that step
    bool rhs_valid = false;
    double rhs_al2s = 0.0;
    double* omega = nullptr; // Chebyshev weights (device, relax_max_iter + 2)
    double gauss_kappa = 0.0; // damping of the Gauss-law filter: 1 / max |K|^2
    // time step of the particle and field kernels: kick (momentum update) and drift
    // (positions, current, fields); both dt except inside a composed step
    double dt_kick = 0.0, dt_drift = 0.0;
    double drift_ratio = 1.0;  // next drift / this drift (where the split form stores a particle)
    // relaxation constants per drift size: [0] for dt, [1] and [2] for the two drifts of
    // the fourth-order composition; the fields above hold the active set
    struct RelaxSet {
        double drift = 0.0, diagA = 1.0, jac_rho = 0.0, gamma = 1.0, r = 0.0, bound = 0.0;
        int sweeps = 0;
        bool converged = true;
        double* omega = nullptr;
    } rs[3];
    int nrs = 1;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timing = false;
    bool t_pending = false;
    double t_ms = 0.0;
    int64_t t_launches = 0;

    int64_t step = 0;
};

namespace pp {

// the high-order line solve turns the second-order charge-conserving current into the
// field-order one; the direct current is deposited as it is
inline bool uses_line_solve(const pp_run* r) {
    return r->p.field_order > 2 && r->p.current_scheme == PP_CURRENT_CC;
}

// Fourth-order composition (Forest and Ruth 1990, position form): theta = 1/(2 - 2^(1/3));
// substep (kick, drift) factors of dt after merging the half drifts of consecutive steps
constexpr double FR_THETA = 1.3512071919596578;
constexpr double FR_KICK[3] = {FR_THETA, 1.0 - 2.0 * FR_THETA, FR_THETA};
constexpr double FR_DRIFT[3] = {0.5 * (1.0 - FR_THETA), 0.5 * (1.0 - FR_THETA), FR_THETA};
void use_relax_set(pp_run* r, int k);  // make relaxation set k active

void set_hip_error(hipError_t e, const char* where);
void set_error_text(const char* msg);  // a library error message for pp_last_hip_error
inline bool ok(hipError_t e, const char* where) {
    if (e != hipSuccess) {
        set_hip_error(e, where);
        return false;
    }
    return true;
}

// kernels launchers (defined in the kernel translation units)
hipError_t launch_gpd64(pp_run* r, int s, double* J);
hipError_t launch_gpd32(pp_run* r, double* J);
hipError_t launch_line_solve(pp_run* r, const double* J2, double* J);
hipError_t launch_field_step(pp_run* r);
int64_t field_blocks(const pp_run* r);  // blocks of one field launch of this run
// Sort species s: FP64 form, counting sort by cell; split form, the tile order (pairs of
// ranks in chunks of 64) per tile, from the particle kernel's counts and ranks when it has
// run since the last sort, otherwise (first sort, arbitrary order) by bucketing and a
// per-tile rebuild.
hipError_t launch_sort(pp_run* r, int s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
void sort_enqueued(pp_run* r, int s);  // host bookkeeping after a ranked sort was enqueued
// move the particles of species s (or of every species, s = -1) to a pending sort order
hipError_t materialize(pp_run* r, int s);
hipError_t launch_diag(pp_run* r, uint32_t what, double* host_out);
hipError_t deposit_rho_all(pp_run* r);  // rho of the current positions into r->rho
hipError_t launch_gauss_filter(pp_run* r);  // the run's Gauss-law filter passes on E
void note_relax_rhs(pp_run* r);  // R holds the right-hand side of the field step just enqueued
// max |R - A B| and max |R| of the last field step (A = 1 - al2s lap) into acc[0], acc[1]
// (bits of non-negative doubles, combined with atomic max: acc must start at zero)
hipError_t launch_relax_resid(pp_run* r, double* acc);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st);
void swap_buffers(pp_particles& c);

// batched launches (pp_batch.hip builds the descriptor tables)
size_t gpd32_args_size();
size_t gpd32_fixed_desc_size();
bool gpd32_batchable(const pp_run* r);
size_t gpd32_lds_bytes(const pp_run* r);
struct Gpd32Args;
struct FixedDesc;
struct FieldDesc;
struct LineArgs;
struct SortDesc;
void gpd32_fill_args(const pp_run* r, Gpd32Args* A);
void gpd32_fixed_desc(const pp_run* r, double* J, FixedDesc* D);
hipError_t launch_gpd32_batch(const void* args_table, const int64_t* tile_prefix, int64_t total_tiles,
                              const void* fixed_table, const int64_t* fixed_prefix, int64_t total_fixed_blocks, int n,
                              int shape_order, size_t lds, hipStream_t st);
size_t field_desc_size();
void field_desc(const pp_run* r, FieldDesc* D);
hipError_t launch_field_step_batch(const void* table, const int64_t* prefix, int n, int64_t total_blocks,
                                   int max_sweeps, hipStream_t st);
size_t line_desc_size();
int64_t line_blocks(const pp_run* r);  // blocks of one line-solve launch of this run
void line_desc(const pp_run* r, const double* J2, double* J, LineArgs* A);
hipError_t launch_line_solve_batch(const void* table, const int64_t* prefix, int n, int64_t total_blocks, hipStream_t st);
size_t sort_desc_size();
void sort_desc(const pp_run* r, int s, SortDesc* D);
constexpr int SORT_BATCH_PHASES = 4;
void sort_desc_blocks(const pp_run* r, int s, int64_t blocks[SORT_BATCH_PHASES]);
hipError_t launch_sort_batch(const void* table, const int64_t* const prefixes[SORT_BATCH_PHASES],
                             const int64_t totals[SORT_BATCH_PHASES], int nseg, hipStream_t st);

}  // namespace pp
