// C ABI of libpp (include/pp.h): validation, run state, launch sequencing.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "pp_internal.hpp"

namespace pp {

static std::mutex g_err_mu;
static char g_err[256] = "";

void set_hip_error(hipError_t e, const char* where) {
    std::lock_guard<std::mutex> lk(g_err_mu);
    snprintf(g_err, sizeof(g_err), "%s: %s", where, hipGetErrorString(e));
}

void set_error_text(const char* msg) {
    std::lock_guard<std::mutex> lk(g_err_mu);
    snprintf(g_err, sizeof(g_err), "%s", msg);
}

// defined in the kernel translation units
hipError_t field_setup(pp_run* r);
int line_setup_axis(int order, int N, double* coef_host, int* off);
int64_t scan_tmp_size(int64_t n);
int diag_acc_count();
size_t gpd32_lds_bytes(const pp_run* r);

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

static pp_status validate(const pp_params* p) {
    if (!p) return PP_E_ARG;
    for (int d = 0; d < 3; ++d) {
        if (p->n[d] < 1 || p->n[d] > (1 << 20)) return PP_E_ARG;
        if (!std::isfinite(p->d[d])) return PP_E_NONFINITE;
        if (!(p->d[d] > 0.0)) return PP_E_ARG;
    }
    const int64_t nc = (int64_t)p->n[0] * p->n[1] * p->n[2];
    if (nc > ((int64_t)1 << 30)) return PP_E_CAPACITY;
    if (!std::isfinite(p->dt) || !std::isfinite(p->c) || !std::isfinite(p->eps0) || !std::isfinite(p->alpha) ||
        !std::isfinite(p->relax_tol) || !std::isfinite(p->rho_background) || !std::isfinite(p->rad_tau))
        return PP_E_NONFINITE;
    if (p->rad_tau < 0.0) return PP_E_ARG;
    if (p->current_scheme != PP_CURRENT_CC && p->current_scheme != PP_CURRENT_DIRECT) return PP_E_ARG;
    if (p->gauss_filter_passes < 0 || p->gauss_filter_passes > PP_MAX_GAUSS_PASSES) return PP_E_ARG;
    if (p->time_order != 2 && p->time_order != 4) return PP_E_ARG;
    if (p->gauss_filter_every < 0 || p->gauss_filter_every > (1 << 20)) return PP_E_ARG;
    if (p->gauss_filter_every > 1 && p->time_order != 2) return PP_E_ARG;
    if (!finite_pos(p->dt) || !finite_pos(p->c) || !finite_pos(p->eps0)) return PP_E_ARG;
    if (p->shape_order != 2 && p->shape_order != 3) return PP_E_ARG;
    if (p->field_order != 2 && p->field_order != 4 && p->field_order != 6) return PP_E_ARG;
    if (!(p->alpha >= 0.5 && p->alpha < 1.0)) return PP_E_ARG;
    if (p->pusher != PP_PUSH_VAY && p->pusher != PP_PUSH_BORIS) return PP_E_ARG;
    if (p->precision != PP_PREC_FP64 && p->precision != PP_PREC_FP32_SPLIT) return PP_E_ARG;
    if (!(p->relax_tol > 0.0 && p->relax_tol < 1.0) || p->relax_max_iter < 1) return PP_E_ARG;
    double dmin = p->d[0];
    for (int d = 1; d < 3; ++d) dmin = p->d[d] < dmin ? p->d[d] : dmin;
    if (!(p->c * p->dt < dmin)) return PP_E_CFL;
    if (p->time_order == 4 && !(FR_THETA * p->c * p->dt < dmin)) return PP_E_CFL;  // the longest drift
    return PP_OK;
}

// Tile shape: powers of two with product TILE_CELLS where the box allows, as close to a cube
// as the box allows (the LDS halo per cell is smallest for a cube): double the shortest tile
// side that is still below the box side.  Boxes at least 4 cells on every side get 4x4x4
// tiles, flat boxes 8x8x1.
static void choose_tiles(const int n[3], int t[3]) {
    t[0] = t[1] = t[2] = 1;
    while (t[0] * t[1] * t[2] < TILE_CELLS) {
        int best = -1;
        for (int d = 0; d < 3; ++d)
            if (t[d] < n[d] && (best < 0 || t[d] < t[best])) best = d;
        if (best < 0) break;
        t[best] *= 2;
    }
}

template <typename T>
static bool dmalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return ok(hipMalloc((void**)p, count * sizeof(T)), "hipMalloc");
}

static void release(pp_run* r) {
    auto f = [](void* p) {
        if (p) (void)hipFree(p);
    };
    f(r->J2);
    f(r->Bn);
    f(r->Bw);
    f(r->R);
    f(r->rho);
    f(r->rho_prev);
    f(r->sort_cursor);
    f(r->sort_scratch);
    f(r->scan_tmp);
    f(r->flags);
    f(r->dacc);
    f(r->Jq);
    f(r->tile_max);
    f(r->qscale);
    for (auto& S : r->rs) f(S.omega);
    f(r->rounds);
    for (int s = 0; s < PP_MAX_SPECIES; ++s) {
        f(r->sp[s].cell_cnt);
        f(r->sp[s].rank);
        f(r->sp[s].perm);
        f(r->sp[s].offsets_next);
    }
    for (int d = 0; d < 3; ++d) f(r->line[d].coef);
    for (int s = 0; s < PP_MAX_SPECIES; ++s) f(r->sp[s].offsets);
    if (r->ev0) (void)hipEventDestroy(r->ev0);
    if (r->ev1) (void)hipEventDestroy(r->ev1);
}

static pp_status flush_timing(pp_run* r) {
    if (!r->timing || !r->t_pending) return PP_OK;
    if (!ok(hipEventSynchronize(r->ev1), "hipEventSynchronize")) return PP_E_HIP;
    float ms = 0.f;
    if (!ok(hipEventElapsedTime(&ms, r->ev0, r->ev1), "hipEventElapsedTime")) return PP_E_HIP;
    r->t_ms += ms;
    r->t_launches += 1;
    r->t_pending = false;
    return PP_OK;
}

}  // namespace pp

using namespace pp;

extern "C" {

const char* pp_status_str(pp_status st) {
    switch (st) {
    case PP_OK: return "ok";
    case PP_E_ARG: return "invalid argument";
    case PP_E_CFL: return "c*dt must be below the smallest cell size";
    case PP_E_NONFINITE: return "non-finite parameter";
    case PP_E_NOCONV: return "field relaxation did not converge";
    case PP_E_CAPACITY: return "size limit exceeded";
    case PP_E_HIP: return "HIP runtime error";
    case PP_E_STATE: return "call order violated";
    default: return "unknown status";
    }
}

const char* pp_last_hip_error(void) { return g_err; }

// Device bytes pp_create and pp_init_species allocate for a run (the caller-owned mesh and
// particle arrays not included); mirrors the allocations below.
static size_t internal_bytes(const pp_params* p, const Geom& g, int64_t nmax, int nsp) {
    const size_t nc = (size_t)g.ncell, n3 = 3 * nc, nb = (size_t)g.nbins;
    size_t b = 0;
    if (p->field_order > 2) b += n3 * sizeof(double);                     // J2
    b += 3 * n3 * sizeof(double);                                          // Bn, Bw, R
    b += 2 * nc * sizeof(double);                                          // rho, rho_prev
    b += nb * sizeof(int32_t) + (size_t)scan_tmp_size(g.nbins + 1) * sizeof(int32_t);
    b += sizeof(int32_t) + ((size_t)diag_acc_count() + 8) * sizeof(double);
    b += (p->time_order == 4 ? 3 : 1) * ((size_t)p->relax_max_iter + 2) * sizeof(double);  // relaxation weights
    if (p->precision == PP_PREC_FP32_SPLIT) {
        b += n3 * sizeof(long long) + PP_MAX_SPECIES * sizeof(int32_t) + sizeof(double);
        b += 2 * (size_t)nmax * sizeof(int32_t);                           // sort scratch
        b += (size_t)g.ntiles * SORT_RCAP * sizeof(RoundEntry);            // round tables
        // per species: cell counts, particle ranks and sort permutation, next tile starts
        b += (size_t)nsp * (nc * sizeof(int32_t) + 2 * (size_t)nmax * sizeof(int32_t) +
                            ((size_t)g.ntiles + 1) * sizeof(int32_t));
    }
    if (p->field_order > 2)  // line-solve coefficients: at most min(N, 127) per axis
        for (int d = 0; d < 3; ++d) b += (size_t)(p->n[d] < 127 ? p->n[d] : 127) * sizeof(double);
    b += (size_t)nsp * (nb + 1) * sizeof(int32_t);                        // per-species offsets
    return b;
}

static void make_geom_host(const pp_params* p, Geom& g) {
    for (int d = 0; d < 3; ++d) g.n[d] = p->n[d];
    choose_tiles(g.n, g.t);
    for (int d = 0; d < 3; ++d) g.nt[d] = (g.n[d] + g.t[d] - 1) / g.t[d];
    g.ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    g.ntiles = (int64_t)g.nt[0] * g.nt[1] * g.nt[2];
    g.nbins = g.ntiles * TILE_CELLS;
}

pp_status pp_workspace_size(const pp_params* params, int64_t max_particles, int32_t nspecies, size_t* bytes) {
    if (!bytes) return PP_E_ARG;
    *bytes = 0;
    pp_status st = validate(params);
    if (st != PP_OK) return st;
    if (max_particles < 0 || nspecies < 0 || nspecies > PP_MAX_SPECIES) return PP_E_ARG;
    if (max_particles >= INT32_MAX) return PP_E_CAPACITY;
    Geom g;
    make_geom_host(params, g);
    if (g.nbins + 1 > INT32_MAX) return PP_E_CAPACITY;
    *bytes = internal_bytes(params, g, max_particles, nspecies);
    return PP_OK;
}

pp_status pp_create(const pp_params* params, const pp_mesh* mesh, void* hip_stream, pp_run** out) {
    if (!out) return PP_E_ARG;
    *out = nullptr;
    pp_status st = validate(params);
    if (st != PP_OK) return st;
    if (!mesh || !mesh->E || !mesh->B || !mesh->J) return PP_E_ARG;
    pp_run* r = new (std::nothrow) pp_run();
    if (!r) return PP_E_CAPACITY;
    r->p = *params;
    r->mesh = *mesh;
    r->stream = (hipStream_t)hip_stream;
    Geom& g = r->g;
    make_geom_host(params, g);
    if (g.nbins + 1 > INT32_MAX) {
        delete r;
        return PP_E_CAPACITY;
    }
    const size_t n3 = 3 * (size_t)g.ncell;
    bool okk = true;
    if (params->field_order > 2) okk = okk && dmalloc(&r->J2, n3);
    okk = okk && dmalloc(&r->Bn, n3) && dmalloc(&r->Bw, n3) && dmalloc(&r->R, n3);
    okk = okk && dmalloc(&r->rho, (size_t)g.ncell) && dmalloc(&r->rho_prev, (size_t)g.ncell);
    okk = okk && dmalloc(&r->sort_cursor, (size_t)g.nbins) && dmalloc(&r->scan_tmp, (size_t)scan_tmp_size(g.nbins + 1));
    okk = okk && dmalloc(&r->flags, 1) && dmalloc(&r->dacc, (size_t)diag_acc_count() + 8);
    r->nrs = params->time_order == 4 ? 3 : 1;
    for (int k = 0; k < r->nrs; ++k) okk = okk && dmalloc(&r->rs[k].omega, (size_t)params->relax_max_iter + 2);
    if (params->precision == PP_PREC_FP32_SPLIT) {
        okk = okk && dmalloc(&r->rounds, (size_t)g.ntiles * SORT_RCAP);
        okk = okk && dmalloc(&r->Jq, n3) && dmalloc(&r->tile_max, PP_MAX_SPECIES) && dmalloc(&r->qscale, 1) &&
              ok(hipMemset(r->tile_max, 0, PP_MAX_SPECIES * sizeof(int32_t)), "hipMemset");
    }
    if (okk && params->field_order > 2) {
        for (int d = 0; d < 3; ++d) {
            double host[1024 + 128];
            int off = 0;
            const int N = g.n[d];
            // the full circulant is used on short lines; long lines use a truncated stencil
            double* buf = host;
            double* heap = nullptr;
            if (N > 1024) {
                heap = new (std::nothrow) double[N];
                if (!heap) {
                    okk = false;
                    break;
                }
                buf = heap;
            }
            int len = line_setup_axis(params->field_order, N, buf, &off);
            r->line[d].len = len;
            r->line[d].off = off;
            okk = okk && dmalloc(&r->line[d].coef, (size_t)len) &&
                  ok(hipMemcpy(r->line[d].coef, buf, len * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
            delete[] heap;
        }
    }
    okk = okk && ok(hipMemset(r->flags, 0, sizeof(int32_t)), "hipMemset");
    okk = okk && ok(hipEventCreate(&r->ev0), "hipEventCreate") && ok(hipEventCreate(&r->ev1), "hipEventCreate");
    if (okk && params->precision == PP_PREC_FP32_SPLIT) {
        int dev = 0;
        hipDeviceProp_t prop;
        okk = ok(hipGetDevice(&dev), "hipGetDevice") && ok(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
        if (okk && gpd32_lds_bytes(r) > (size_t)prop.sharedMemPerBlock) {
            release(r);
            delete r;
            return PP_E_CAPACITY;
        }
    }
    if (!okk) {
        release(r);
        delete r;
        return PP_E_HIP;
    }
    if (!ok(field_setup(r), "field_setup")) {
        release(r);
        delete r;
        return PP_E_HIP;
    }
    *out = r;
    return PP_OK;
}

pp_status pp_init_species(pp_run* r, int32_t s, double q, double m, double w, const pp_particles* parts) {
    if (!r || !parts || s < 0 || s >= PP_MAX_SPECIES) return PP_E_ARG;
    if (!std::isfinite(q) || !std::isfinite(m) || !std::isfinite(w)) return PP_E_NONFINITE;
    if (!(m > 0.0) || w < 0.0) return PP_E_ARG;
    if (parts->n < 0 || parts->n >= INT32_MAX) return PP_E_CAPACITY;
    const bool split = r->p.precision == PP_PREC_FP32_SPLIT;
    if (parts->n > 0) {
        for (int d = 0; d < 3; ++d)
            if (!parts->pos[d] || !parts->u[d] || !parts->pos_alt[d] || !parts->u_alt[d]) return PP_E_ARG;
        if (split && (!parts->cell || !parts->cell_alt)) return PP_E_ARG;
        if (parts->id && !parts->id_alt) return PP_E_ARG;
    }
    Species& S = r->sp[s];
    if (!S.offsets && !dmalloc(&S.offsets, (size_t)r->g.nbins + 1)) return PP_E_HIP;
    if (split) {
        if (!S.offsets_next && !dmalloc(&S.offsets_next, (size_t)r->g.ntiles + 1)) return PP_E_HIP;
        if (!S.cell_cnt && !dmalloc(&S.cell_cnt, (size_t)r->g.ncell)) return PP_E_HIP;
        if (!ok(launch_fill_i32(S.cell_cnt, r->g.ncell, 0, r->stream), "fill")) return PP_E_HIP;
        if (S.rank) (void)hipFree(S.rank);
        S.rank = nullptr;
        if (!dmalloc(&S.rank, (size_t)parts->n)) return PP_E_HIP;
        if (S.perm) (void)hipFree(S.perm);
        S.perm = nullptr;
        if (!dmalloc(&S.perm, (size_t)parts->n)) return PP_E_HIP;
    }
    S.pending = false;
    if (split && parts->n > r->sort_scratch_n) {
        if (r->sort_scratch) (void)hipFree(r->sort_scratch);
        r->sort_scratch = nullptr;
        r->sort_scratch_n = 0;
        if (!dmalloc(&r->sort_scratch, 2 * (size_t)parts->n)) return PP_E_HIP;
        r->sort_scratch_n = parts->n;
    }
    S.active = true;
    S.q = q;
    S.m = m;
    S.w = w;
    S.n = parts->n;
    S.cur = *parts;
    if (!split) {
        S.cur.cell = nullptr;
        S.cur.cell_alt = nullptr;
    }
    if (!parts->id) S.cur.id_alt = nullptr;
    S.sorted = false;
    S.ranked = false;
    // initial sort: the split form needs it before its first push
    hipError_t e = launch_sort(r, s);
    if (!ok(e, "sort")) return PP_E_HIP;
    return PP_OK;
}

pp_status pp_gather_push_deposit(pp_run* r) {
    if (!r) return PP_E_ARG;
    const bool split = r->p.precision == PP_PREC_FP32_SPLIT;
    for (int s = 0; s < PP_MAX_SPECIES; ++s)
        if (split && r->sp[s].active && !r->sp[s].sorted) return PP_E_STATE;
    if (flush_timing(r) != PP_OK) return PP_E_HIP;
    double* target = uses_line_solve(r) ? r->J2 : r->mesh.J;
    hipError_t e = hipSuccess;
    if (!split) {  // the split kernel overwrites its target
        e = launch_fill(target, 3 * r->g.ncell, 0.0, r->stream);
        if (!ok(e, "fill")) return PP_E_HIP;
    }
    if (r->timing && !ok(hipEventRecord(r->ev0, r->stream), "hipEventRecord")) return PP_E_HIP;
    if (split) {
        e = launch_gpd32(r, target);
        if (!ok(e, "gather_push_deposit")) return PP_E_HIP;
        for (int s = 0; s < PP_MAX_SPECIES; ++s) {  // the kernel wrote the pending order
            Species& S = r->sp[s];
            if (!S.active || !S.pending) continue;
            swap_buffers(S.cur);
            S.pending = false;
        }
    } else {
        for (int s = 0; s < PP_MAX_SPECIES; ++s) {
            if (!r->sp[s].active) continue;
            e = launch_gpd64(r, s, target);
            if (!ok(e, "gather_push_deposit")) return PP_E_HIP;
        }
    }
    if (r->timing) {
        if (!ok(hipEventRecord(r->ev1, r->stream), "hipEventRecord")) return PP_E_HIP;
        r->t_pending = true;
    }
    for (int s = 0; s < PP_MAX_SPECIES; ++s)
        if (split && r->sp[s].active) {
            r->sp[s].sorted = false;
            r->sp[s].ranked = true;  // the kernel counted the new cells for the next sort
        }
    if (uses_line_solve(r)) {
        e = launch_line_solve(r, r->J2, r->mesh.J);
        if (!ok(e, "line_solve")) return PP_E_HIP;
    }
    r->step += 1;
    return PP_OK;
}

pp_status pp_field_step(pp_run* r) {
    if (!r) return PP_E_ARG;
    hipError_t e = launch_field_step(r);
    if (!ok(e, "field_step")) return PP_E_HIP;
    const int every = r->p.gauss_filter_every;
    if (r->p.gauss_filter_passes > 0 && (every <= 1 || r->step % every == 0)) {
        e = launch_gauss_filter(r);
        if (!ok(e, "gauss_filter")) return PP_E_HIP;
    }
    // the step is done either way; relax_max_iter sweeps could not reach relax_tol
    return r->jac_converged ? PP_OK : PP_E_NOCONV;
}

pp_status pp_step(pp_run* r) {
    if (!r) return PP_E_ARG;
    if (r->p.time_order != 4) {
        pp_status st = pp_gather_push_deposit(r);
        if (st == PP_OK) st = pp_sort_particles(r, -1);
        if (st == PP_OK) st = pp_field_step(r);
        return st;
    }
    pp_status st = PP_OK;
    bool noconv = false;  // a substep's relaxation capped: the step still completes
    for (int k = 0; k < 3 && st == PP_OK; ++k) {
        use_relax_set(r, k < 2 ? 1 : 2);  // sets 1 and 2 hold the drifts (1-theta)/2 dt and theta dt
        r->dt_kick = FR_KICK[k] * r->p.dt;
        r->drift_ratio = FR_DRIFT[(k + 1) % 3] / FR_DRIFT[k];
        st = pp_gather_push_deposit(r);
        if (st == PP_OK) st = pp_sort_particles(r, -1);
        if (st == PP_OK) st = pp_field_step(r);
        if (st == PP_E_NOCONV) {
            noconv = true;
            st = PP_OK;
        }
    }
    use_relax_set(r, 0);
    r->dt_kick = r->p.dt;
    r->drift_ratio = 1.0;
    r->step -= 2;             // one step, three particle substeps
    r->rho_prev_step = -1;    // J is the last substep's: no continuity check across the step
    return st == PP_OK && noconv ? PP_E_NOCONV : st;
}

pp_status pp_sort_particles(pp_run* r, int32_t s) {
    if (!r || s < -1 || s >= PP_MAX_SPECIES) return PP_E_ARG;
    for (int k = 0; k < PP_MAX_SPECIES; ++k) {
        if (s >= 0 && k != s) continue;
        if (!r->sp[k].active) {
            if (s >= 0) return PP_E_STATE;
            continue;
        }
        hipError_t e = launch_sort(r, k);
        if (!ok(e, "sort")) return PP_E_HIP;
    }
    return PP_OK;
}

pp_status pp_diagnostics(pp_run* r, uint32_t what, pp_diag* out) {
    if (!r || !out) return PP_E_ARG;
    double host[64];
    const int na = diag_acc_count();
    hipError_t e = launch_diag(r, what, host);
    if (!ok(e, "diagnostics")) return PP_E_HIP;
    std::memset(out, 0, sizeof(*out));
    for (int s = 0; s < PP_MAX_SPECIES; ++s) {
        out->kinetic[s] = host[s];
        for (int d = 0; d < 3; ++d) out->momentum[s][d] = host[PP_MAX_SPECIES + 3 * s + d];
    }
    const int base = 4 * PP_MAX_SPECIES;
    out->field_E = host[base + 0];
    out->field_B = host[base + 1];
    out->field_Ex = host[base + 2];
    out->gauss_max = host[base + 3];
    const bool have_prev = host[na + 1] != 0.0;
    out->cc_max = have_prev ? host[base + 4] : NAN;
    out->divB_max = host[base + 5];
    const bool have_relax = host[na + 2] != 0.0;
    out->relax_resid_meas = have_relax ? (host[base + 7] > 0.0 ? host[base + 6] / host[base + 7] : host[base + 6]) : NAN;
    double rref = 0.0;
    const double V = 1.0;
    (void)V;
    for (int s = 0; s < PP_MAX_SPECIES; ++s) {
        const Species& S = r->sp[s];
        if (!S.active) continue;
        // mean number density n_s = w N_s / N_cells
        double ns = S.w * (double)S.n / (double)r->g.ncell;
        double v = std::fabs(S.q) * ns;
        if (v > rref) rref = v;
    }
    out->rho_ref = rref;
    out->relax_resid = r->jac_bound;
    out->relax_iters = r->jac_sweeps;
    out->flags = (int32_t)host[na];
    out->step = r->step;
    return PP_OK;
}

pp_status pp_get_particles(pp_run* r, int32_t s, pp_particles* out) {
    if (!r || !out || s < 0 || s >= PP_MAX_SPECIES) return PP_E_ARG;
    if (!r->sp[s].active) return PP_E_STATE;
    if (!ok(materialize(r, s), "materialize")) return PP_E_HIP;  // the buffers in sort order
    *out = r->sp[s].cur;
    return PP_OK;
}

pp_status pp_timing_enable(pp_run* r, int32_t enable) {
    if (!r) return PP_E_ARG;
    if (flush_timing(r) != PP_OK) return PP_E_HIP;
    r->timing = enable != 0;
    return PP_OK;
}

pp_status pp_timing_read(pp_run* r, double* ms_total, int64_t* launches) {
    if (!r || !ms_total || !launches) return PP_E_ARG;
    if (flush_timing(r) != PP_OK) return PP_E_HIP;
    *ms_total = r->t_ms;
    *launches = r->t_launches;
    r->t_ms = 0.0;
    r->t_launches = 0;
    return PP_OK;
}

pp_status pp_destroy(pp_run* r) {
    if (!r) return PP_E_ARG;
    if (r->stream) (void)hipStreamSynchronize(r->stream);
    else (void)hipDeviceSynchronize();
    release(r);
    delete r;
    return PP_OK;
}

}  // extern "C"
