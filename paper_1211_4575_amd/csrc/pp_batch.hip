// Continuous batching of many small runs: a pp_batch holds a set of runs (each with its own
// mesh, particles and scratch) and steps all of them together, each phase of the step being
// one launch over every member run.  Runs join and leave between steps, so requests that
// arrive while others are running are admitted as soon as there is room.  The batched
// kernels run the same per-tile / per-cell bodies as the single-run launches, and every
// reduction in the step is exact (integer) or fixed-order, so a run's results do not depend
// on which other runs share its launches.
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "pp_internal.hpp"

namespace pp {
void sort_desc(const pp_run* r, int s, SortDesc* D);
}  // namespace pp

struct pp_batch {
    hipStream_t stream = nullptr;
    int device = 0;  // the GPU current at pp_batch_create (its static table array is used)
    int max_runs = 0;
    std::vector<pp_run*> runs;
    // per-step index lists, reserved for max_runs entries at creation (a step never grows them)
    std::vector<int> line_runs;
    std::vector<int> slot_segs[PP_MAX_SPECIES];
    unsigned char* d_buf = nullptr;  // device copy of the step's descriptor tables
    size_t d_cap = 0;
    unsigned char* h_buf[2] = {nullptr, nullptr};  // pinned staging, used alternately
    size_t h_cap = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool ev_used[2] = {false, false};
    int which = 0;
};

// Descriptor tables of pp_batch_step_noalloc: one fixed array per GPU for the life of the
// process, shared by every batch on that GPU.  Host code never passes its name to a kernel or
// a copy (on the host it is only a stand-in): it uses the device address obtained once per
// device by table_array_setup.
static __device__ __align__(256) unsigned char scratch[PP_BATCH_NOALLOC_TABLE_BYTES];

namespace {

using namespace pp;

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    }
};

constexpr int MAX_DEVICES = 64;
std::mutex g_table_mu;
unsigned char* g_table_ptr[MAX_DEVICES] = {};  // device address of `scratch` per GPU

// Device address of the static table array on GPU `dev`, which must be the current device.
pp_status table_array_setup(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) return PP_E_CAPACITY;
    std::lock_guard<std::mutex> lk(g_table_mu);
    if (g_table_ptr[dev]) return PP_OK;
    void* ptr = nullptr;
    if (!ok(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress")) return PP_E_HIP;
    g_table_ptr[dev] = (unsigned char*)ptr;
    return PP_OK;
}

unsigned char* table_array(int dev) {
    std::lock_guard<std::mutex> lk(g_table_mu);
    return dev >= 0 && dev < MAX_DEVICES ? g_table_ptr[dev] : nullptr;
}

// Pinned staging of at least `need` bytes (both halves).
pp_status grow_host(pp_batch* b, size_t need) {
    if (need <= b->h_cap) return PP_OK;
    const size_t cap = need * 2;
    for (int i = 0; i < 2; ++i) {
        if (b->ev_used[i]) (void)hipEventSynchronize(b->ev[i]);
        if (b->h_buf[i]) (void)hipHostFree(b->h_buf[i]);
        b->h_buf[i] = nullptr;
        b->ev_used[i] = false;
    }
    b->h_cap = 0;
    for (int i = 0; i < 2; ++i)
        if (!ok(hipHostMalloc((void**)&b->h_buf[i], cap, hipHostMallocDefault), "hipHostMalloc")) return PP_E_HIP;
    b->h_cap = cap;
    return PP_OK;
}

// The batch's own device table buffer of at least `need` bytes.
pp_status grow_device(pp_batch* b, size_t need) {
    if (need <= b->d_cap) return PP_OK;
    const size_t cap = need * 2;
    if (b->d_buf) {
        (void)hipStreamSynchronize(b->stream);
        (void)hipFree(b->d_buf);
    }
    b->d_buf = nullptr;
    b->d_cap = 0;
    if (!ok(hipMalloc((void**)&b->d_buf, cap), "hipMalloc")) return PP_E_HIP;
    b->d_cap = cap;
    return PP_OK;
}

enum TableTarget { TABLES_OWN = 0, TABLES_STATIC = 1 };

// One step of every member (the body of pp_batch_step and pp_batch_step_noalloc).  With
// TABLES_OWN the batch's buffers grow as needed; with TABLES_STATIC nothing is allocated: the
// tables go to the GPU's static array through the pinned staging made by pp_batch_create.
pp_status batch_step(pp_batch* b, TableTarget target) {
    const int n = (int)b->runs.size();
    if (n == 0) return PP_OK;
    for (pp_run* r : b->runs)
        for (int s = 0; s < PP_MAX_SPECIES; ++s)
            if (r->sp[s].active && !r->sp[s].sorted) return PP_E_STATE;

    // ---- layout of the step's descriptor tables --------------------------------------
    std::vector<int>& line_runs = b->line_runs;
    line_runs.clear();
    for (int i = 0; i < n; ++i)
        if (uses_line_solve(b->runs[i])) line_runs.push_back(i);
    const int nl = (int)line_runs.size();
    std::vector<int>* slot_segs = b->slot_segs;
    for (int s = 0; s < PP_MAX_SPECIES; ++s) {
        slot_segs[s].clear();
        for (int i = 0; i < n; ++i)
            if (b->runs[i]->sp[s].active) slot_segs[s].push_back(i);
    }

    Layout L;
    const size_t o_gpd = L.take(n * gpd32_args_size());
    const size_t o_tpre = L.take((n + 1) * sizeof(int64_t));
    const size_t o_fix = L.take(n * gpd32_fixed_desc_size());
    const size_t o_fpre = L.take((n + 1) * sizeof(int64_t));
    const size_t o_line = L.take((nl + 1) * line_desc_size());
    const size_t o_lpre = L.take((nl + 1) * sizeof(int64_t));
    size_t o_sort[PP_MAX_SPECIES], o_spre[PP_MAX_SPECIES][SORT_BATCH_PHASES];
    for (int s = 0; s < PP_MAX_SPECIES; ++s) {
        const int ns = (int)slot_segs[s].size();
        o_sort[s] = L.take((ns + 1) * sort_desc_size());
        for (int ph = 0; ph < SORT_BATCH_PHASES; ++ph) o_spre[s][ph] = L.take((ns + 1) * sizeof(int64_t));
    }
    const size_t o_field = L.take(n * field_desc_size());
    const size_t o_cpre = L.take((n + 1) * sizeof(int64_t));
    unsigned char* D = nullptr;
    if (target == TABLES_OWN) {
        if (grow_host(b, L.off) != PP_OK || grow_device(b, L.off) != PP_OK) return PP_E_HIP;
        D = b->d_buf;
    } else {
        if (L.off > (size_t)PP_BATCH_NOALLOC_TABLE_BYTES || L.off > b->h_cap) {
            char msg[160];
            snprintf(msg, sizeof msg, "pp_batch_step_noalloc: the step's tables need %zu bytes, above the static %d",
                     L.off, (int)PP_BATCH_NOALLOC_TABLE_BYTES);
            set_error_text(msg);
            return PP_E_CAPACITY;
        }
        D = table_array(b->device);
        if (!D) {
            set_error_text("pp_batch_step_noalloc: no static table array on this batch's GPU");
            return PP_E_STATE;
        }
    }

    const int w = b->which;
    if (b->ev_used[w] && !ok(hipEventSynchronize(b->ev[w]), "hipEventSynchronize")) return PP_E_HIP;
    unsigned char* H = b->h_buf[w];
    std::memset(H, 0, L.off);
    // ---- fill ------------------------------------------------------------------------
    int64_t* tpre = (int64_t*)(H + o_tpre);
    int64_t* fpre = (int64_t*)(H + o_fpre);
    int64_t* cpre = (int64_t*)(H + o_cpre);
    tpre[0] = fpre[0] = cpre[0] = 0;
    int max_sweeps = 0;
    for (int i = 0; i < n; ++i) {
        pp_run* r = b->runs[i];
        double* target = uses_line_solve(r) ? r->J2 : r->mesh.J;
        gpd32_fill_args(r, (Gpd32Args*)(H + o_gpd + i * gpd32_args_size()));
        for (int s = 0; s < PP_MAX_SPECIES; ++s) {  // the kernel writes the pending order
            Species& S = r->sp[s];
            if (!S.active || !S.pending) continue;
            swap_buffers(S.cur);
            S.pending = false;
        }
        gpd32_fixed_desc(r, target, (FixedDesc*)(H + o_fix + i * gpd32_fixed_desc_size()));
        field_desc(r, (FieldDesc*)(H + o_field + i * field_desc_size()));
        tpre[i + 1] = tpre[i] + r->g.ntiles;
        fpre[i + 1] = fpre[i] + (3 * r->g.ncell + 255) / 256;
        cpre[i + 1] = cpre[i] + field_blocks(r);
        max_sweeps = r->jac_sweeps > max_sweeps ? r->jac_sweeps : max_sweeps;
    }
    int64_t* lpre = (int64_t*)(H + o_lpre);
    lpre[0] = 0;
    for (int j = 0; j < nl; ++j) {
        pp_run* r = b->runs[line_runs[j]];
        line_desc(r, r->J2, r->mesh.J, (LineArgs*)(H + o_line + j * line_desc_size()));
        lpre[j + 1] = lpre[j] + line_blocks(r);
    }
    int64_t stot[PP_MAX_SPECIES][SORT_BATCH_PHASES];
    for (int s = 0; s < PP_MAX_SPECIES; ++s) {
        const int ns = (int)slot_segs[s].size();
        int64_t* pre[SORT_BATCH_PHASES];
        for (int ph = 0; ph < SORT_BATCH_PHASES; ++ph) {
            pre[ph] = (int64_t*)(H + o_spre[s][ph]);
            pre[ph][0] = 0;
        }
        for (int j = 0; j < ns; ++j) {
            const int i = slot_segs[s][j];
            sort_desc(b->runs[i], s, (SortDesc*)(H + o_sort[s] + j * sort_desc_size()));
            int64_t blocks[SORT_BATCH_PHASES];
            sort_desc_blocks(b->runs[i], s, blocks);
            for (int ph = 0; ph < SORT_BATCH_PHASES; ++ph) pre[ph][j + 1] = pre[ph][j] + blocks[ph];
        }
        for (int ph = 0; ph < SORT_BATCH_PHASES; ++ph) stot[s][ph] = pre[ph][ns];
    }

    // ---- upload and launch -------------------------------------------------------------
    if (!ok(hipMemcpyAsync(D, H, L.off, hipMemcpyHostToDevice, b->stream), "hipMemcpyAsync")) return PP_E_HIP;
    if (!ok(hipEventRecord(b->ev[w], b->stream), "hipEventRecord")) return PP_E_HIP;
    b->ev_used[w] = true;
    b->which ^= 1;
    hipError_t e = launch_gpd32_batch(D + o_gpd, (const int64_t*)(D + o_tpre), tpre[n], D + o_fix,
                                      (const int64_t*)(D + o_fpre), fpre[n], n, b->runs[0]->p.shape_order,
                                      gpd32_lds_bytes(b->runs[0]), b->stream);
    if (!ok(e, "batch gather_push_deposit")) return PP_E_HIP;
    e = launch_line_solve_batch(D + o_line, (const int64_t*)(D + o_lpre), nl, lpre[nl], b->stream);
    if (!ok(e, "batch line_solve")) return PP_E_HIP;
    for (int s = 0; s < PP_MAX_SPECIES; ++s) {
        const int ns = (int)slot_segs[s].size();
        if (ns == 0) continue;
        const int64_t* pre[SORT_BATCH_PHASES];
        for (int ph = 0; ph < SORT_BATCH_PHASES; ++ph) pre[ph] = (const int64_t*)(D + o_spre[s][ph]);
        e = launch_sort_batch(D + o_sort[s], pre, stot[s], ns, b->stream);
        if (!ok(e, "batch sort")) return PP_E_HIP;
    }
    e = launch_field_step_batch(D + o_field, (const int64_t*)(D + o_cpre), n, cpre[n], max_sweeps, b->stream);
    if (!ok(e, "batch field_step")) return PP_E_HIP;

    // ---- host bookkeeping (tile starts and pending orders after the sort) ------------------
    bool noconv = false;
    for (int i = 0; i < n; ++i) {
        pp_run* r = b->runs[i];
        for (int s = 0; s < PP_MAX_SPECIES; ++s)
            if (r->sp[s].active) sort_enqueued(r, s);
        r->step += 1;
        note_relax_rhs(r);
        noconv = noconv || !r->jac_converged;
    }
    // every member stepped; a member's relaxation could not reach its tolerance
    return noconv ? PP_E_NOCONV : PP_OK;
}

}  // namespace

extern "C" {

pp_status pp_batch_create(int32_t max_runs, void* hip_stream, pp_batch** out) {
    if (!out || max_runs < 1 || max_runs > 4096) return PP_E_ARG;
    *out = nullptr;
    pp_batch* b = new (std::nothrow) pp_batch();
    if (!b) return PP_E_CAPACITY;
    b->stream = (hipStream_t)hip_stream;
    b->max_runs = max_runs;
    b->runs.reserve(max_runs);
    b->line_runs.reserve(max_runs);
    for (auto& v : b->slot_segs) v.reserve(max_runs);
    pp_status st = PP_OK;
    if (!ok(hipGetDevice(&b->device), "hipGetDevice")) st = PP_E_HIP;
    for (int i = 0; i < 2 && st == PP_OK; ++i)
        if (!ok(hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming), "hipEventCreate")) st = PP_E_HIP;
    // pinned staging large enough for the static table array, so that pp_batch_step_noalloc
    // never needs to allocate; pp_batch_step grows it further when its tables need more
    for (int i = 0; i < 2 && st == PP_OK; ++i)
        if (!ok(hipHostMalloc((void**)&b->h_buf[i], PP_BATCH_NOALLOC_TABLE_BYTES, hipHostMallocDefault),
                "hipHostMalloc"))
            st = PP_E_HIP;
    if (st == PP_OK) b->h_cap = PP_BATCH_NOALLOC_TABLE_BYTES;
    if (st == PP_OK) st = table_array_setup(b->device);
    if (st != PP_OK) {
        for (int i = 0; i < 2; ++i) {
            if (b->h_buf[i]) (void)hipHostFree(b->h_buf[i]);
            if (b->ev[i]) (void)hipEventDestroy(b->ev[i]);
        }
        delete b;
        return st;
    }
    *out = b;
    return PP_OK;
}

pp_status pp_batch_add(pp_batch* b, pp_run* r) {
    if (!b || !r) return PP_E_ARG;
    if ((int)b->runs.size() >= b->max_runs) return PP_E_CAPACITY;
    for (pp_run* x : b->runs)
        if (x == r) return PP_E_STATE;
    if (r->p.precision != PP_PREC_FP32_SPLIT || !gpd32_batchable(r)) return PP_E_ARG;
    if (r->stream != b->stream) return PP_E_ARG;
    if (r->p.gauss_filter_passes > 0) return PP_E_ARG;  // the filter has no batched form
    if (r->p.time_order != 2) return PP_E_ARG;          // the batch steps leapfrog steps
    if (!b->runs.empty() && b->runs[0]->p.shape_order != r->p.shape_order) return PP_E_ARG;
    for (int s = 0; s < PP_MAX_SPECIES; ++s)
        if (r->sp[s].active && !r->sp[s].sorted) return PP_E_STATE;
    b->runs.push_back(r);
    return PP_OK;
}

pp_status pp_batch_remove(pp_batch* b, pp_run* r) {
    if (!b || !r) return PP_E_ARG;
    for (size_t i = 0; i < b->runs.size(); ++i)
        if (b->runs[i] == r) {
            b->runs.erase(b->runs.begin() + (long)i);
            return PP_OK;
        }
    return PP_E_STATE;
}

pp_status pp_batch_size(const pp_batch* b, int32_t* n) {
    if (!b || !n) return PP_E_ARG;
    *n = (int32_t)b->runs.size();
    return PP_OK;
}

pp_status pp_batch_step(pp_batch* b) {
    if (!b) return PP_E_ARG;
    return batch_step(b, TABLES_OWN);
}

pp_status pp_batch_step_noalloc(pp_batch* b) {
    if (!b) return PP_E_ARG;
    return batch_step(b, TABLES_STATIC);
}

pp_status pp_batch_destroy(pp_batch* b) {
    if (!b) return PP_E_ARG;
    if (b->stream)
        (void)hipStreamSynchronize(b->stream);
    else
        (void)hipDeviceSynchronize();
    for (int i = 0; i < 2; ++i) {
        if (b->h_buf[i]) (void)hipHostFree(b->h_buf[i]);
        if (b->ev[i]) (void)hipEventDestroy(b->ev[i]);
    }
    if (b->d_buf) (void)hipFree(b->d_buf);
    delete b;
    return PP_OK;
}

}  // extern "C"
