// C ABI of batches: independent instances that advance together, one fused
// launch (one block per work item) per kernel kind and polynomial order,
// captured in HIP graphs.  Instances can be attached and detached between steps (the
// serving loop's continuous batching); each keeps its own workspace, state
// and device CG scalars, and its arithmetic is that of dg_rk_step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "abi_types.h"
#include "batch.h"
#include "dg_launch.h"

using namespace dgk;

namespace {

enum ListKind { kCell = 0, kRow, kPwRows, kPwCells, kPwElems, kListCount };

// Launch groups: one per (polynomial order, cell tile height, bracket tile
// height); every kernel kind of a group is one fused launch.
constexpr int kCellShapes[3] = {4, 8, 16};
constexpr int kRowShapes[2] = {8, 16};
constexpr int kShapes = 6;
constexpr int kGroups = kMaxN * kShapes;
static_assert(kGroups <= 32, "group_mask holds one bit per launch group");

int group_of(const Geom& g) {
    const int ci = g.cw == 4 ? 0 : (g.cw == 8 ? 1 : 2);
    const int ri = g.rw == 8 ? 0 : 1;
    return (g.n - 1) * kShapes + ci * 2 + ri;
}

struct GroupShape {
    int n, cw, rw;
};

GroupShape shape_of(int gi) {
    const int n = gi / kShapes + 1, s = gi % kShapes;
    return GroupShape{n, kCellShapes[s / 2], kRowShapes[s % 2]};
}

struct Slot {
    bool used = false;
    const dg_grid* grid = nullptr;
    double* omega = nullptr;
    double dt = 0.0, D = 0.0;
    dg_workspace* ws = nullptr;
    dg_state* st = nullptr;
    bool converged = true;      // every solve of the last step converged
};

struct DevList {
    BatchItem* items = nullptr;
    int cap = 0;
    int count = 0;
};

}  // namespace

struct dg_batch {
    int capacity = 0;
    int device = 0;
    std::vector<Slot> slots;
    BatchInst* d_inst = nullptr;   // device records
    BatchInst* h_inst = nullptr;   // pinned host records
    CgScalars* d_sc = nullptr;     // device CG scalars, one per slot
    CgScalars* h_sc = nullptr;     // pinned: 3 x capacity (2 poll slots + final)
    int* d_counts = nullptr;       // device item counts [n-1][kind]
    int* h_counts = nullptr;       // pinned
    DevList lists[kGroups][kListCount];
    bool lists_dirty = true;
    unsigned group_mask = 0;       // bit gi set if some slot is in launch group gi
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipStream_t cap = nullptr;     // capture stream
    bool use_graphs = true;
    bool graphs_valid = false;
    int fd_flags = 0;              // preconditioner of the members' workspaces (0: none)
    int chunk = 16;                // CG iterations per captured chunk (even)
    hipGraphExec_t g_setup = nullptr, g_finish = nullptr;
    hipGraphExec_t g_chunk[kGroups] = {};   // CG chunk of each launch group
};

namespace {

void destroy_graphs(dg_batch* b) {
    for (hipGraphExec_t* g : {&b->g_setup, &b->g_finish})
        if (*g) { (void)hipGraphExecDestroy(*g); *g = nullptr; }
    for (hipGraphExec_t& g : b->g_chunk)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
    b->graphs_valid = false;
}

ItemList list_of(const dg_batch* b, int gi, int kind) {
    return ItemList{b->lists[gi][kind].items, b->d_counts + gi * kListCount + kind};
}

int grid_of(const dg_batch* b, int gi, int kind) {
    const int c = b->lists[gi][kind].count;
    return c < 1 ? 1 : c;   // one block per item
}

// Rebuild the per-order work lists (instance, local block) on the host and
// upload them.
int rebuild_lists(dg_batch* b, hipStream_t s) {
    std::vector<BatchItem> h[kGroups][kListCount];
    unsigned mask = 0;
    for (int i = 0; i < b->capacity; ++i) {
        const Slot& sl = b->slots[i];
        if (!sl.used) continue;
        const BatchInst& r = b->h_inst[i];
        const int gi = group_of(r.g);
        mask |= 1u << gi;
        const int counts[kListCount] = {r.cell_nblocks, r.row_nblocks, r.nb_rows,
                                        r.nb_cells, r.nb_elems};
        for (int k = 0; k < kListCount; ++k)
            for (int q = 0; q < counts[k]; ++q) h[gi][k].push_back(BatchItem{i, q});
    }
    bool realloc_any = false;
    for (int n = 0; n < kGroups; ++n)
        for (int k = 0; k < kListCount; ++k) {
            DevList& L = b->lists[n][k];
            const int need = (int)h[n][k].size();
            if (need > L.cap) {
                if (L.items) (void)hipFree(L.items);
                L.items = nullptr;
                int cap = L.cap ? L.cap : 256;
                while (cap < need) cap *= 2;
                if (hipMalloc((void**)&L.items, (size_t)cap * sizeof(BatchItem)) != hipSuccess) {
                    (void)hipGetLastError();
                    L.cap = 0;
                    return fail(DG_E_NOMEM, "batch work list allocation failed");
                }
                L.cap = cap;
                realloc_any = true;
            }
            L.count = need;
            b->h_counts[n * kListCount + k] = need;
            if (need)
                HIP_TRY(hipMemcpyAsync(L.items, h[n][k].data(), need * sizeof(BatchItem),
                                       hipMemcpyHostToDevice, s));
        }
    HIP_TRY(hipMemcpyAsync(b->d_counts, b->h_counts, kGroups * kListCount * sizeof(int),
                           hipMemcpyHostToDevice, s));
    // the host vectors above are pageable: make the copies complete
    HIP_TRY(hipStreamSynchronize(s));
    // launch grids follow the item counts: recapture the graphs
    (void)realloc_any;
    destroy_graphs(b);
    b->group_mask = mask;
    b->lists_dirty = false;
    return DG_OK;
}

int enqueue_setup(dg_batch* b, hipStream_t s) {
    for (int gi = 0; gi < kGroups; ++gi) {
        if (!(b->group_mask & (1u << gi))) continue;
        const GroupShape q = shape_of(gi);
        hipError_t e = launch_batch(q.n, q.cw, q.rw, BatchKernel::Mean, b->d_inst,
                                    list_of(b, gi, kPwRows), grid_of(b, gi, kPwRows), s);
        if (e == hipSuccess)
            e = launch_batch(q.n, q.cw, q.rw, BatchKernel::Init, b->d_inst,
                             list_of(b, gi, kCell), grid_of(b, gi, kCell), s);
        if (e != hipSuccess) return hip_fail(e, "batch setup launch");
    }
    return DG_OK;
}

// b->chunk CG iterations of launch group gi.  The groups hold disjoint
// instances, so each advances by its own chunks: a group whose members have
// all converged is no longer replayed while the others iterate.
int enqueue_chunk(dg_batch* b, int gi, hipStream_t s) {
    const GroupShape q = shape_of(gi);
    for (int i = 0; i < b->chunk; ++i) {
        hipError_t e = launch_batch(q.n, q.cw, q.rw, BatchKernel::Dir, b->d_inst,
                                    list_of(b, gi, kCell), grid_of(b, gi, kCell), s);
        if (e == hipSuccess)
            e = launch_batch(q.n, q.cw, q.rw, BatchKernel::Res, b->d_inst,
                             list_of(b, gi, kCell), grid_of(b, gi, kCell), s);
        if (e != hipSuccess) return hip_fail(e, "batch CG launch");
    }
    return DG_OK;
}

int enqueue_finish(dg_batch* b, hipStream_t s) {
    for (int gi = 0; gi < kGroups; ++gi) {
        if (!(b->group_mask & (1u << gi))) continue;
        const GroupShape q = shape_of(gi);
        hipError_t e = launch_batch(q.n, q.cw, q.rw, BatchKernel::Finish, b->d_inst,
                                    list_of(b, gi, kPwCells), grid_of(b, gi, kPwCells), s);
        if (e == hipSuccess)
            e = launch_batch(q.n, q.cw, q.rw, BatchKernel::SubMean, b->d_inst,
                             list_of(b, gi, kPwElems), grid_of(b, gi, kPwElems), s);
        if (e == hipSuccess)
            e = launch_batch(q.n, q.cw, q.rw, BatchKernel::Rhs, b->d_inst,
                             list_of(b, gi, kRow), grid_of(b, gi, kRow), s);
        if (e != hipSuccess) return hip_fail(e, "batch finish launch");
    }
    return DG_OK;
}

template <class Fn>
int capture(dg_batch* b, Fn&& fn, hipGraphExec_t* out) {
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    int rc = fn(b->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc != DG_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    return DG_OK;
}

int ensure_graphs(dg_batch* b) {
    if (b->graphs_valid) return DG_OK;
    destroy_graphs(b);
    int rc = capture(b, [b](hipStream_t s) { return enqueue_setup(b, s); }, &b->g_setup);
    for (int gi = 0; gi < kGroups && rc == DG_OK; ++gi)
        if (b->group_mask & (1u << gi))
            rc = capture(b, [b, gi](hipStream_t s) { return enqueue_chunk(b, gi, s); },
                         &b->g_chunk[gi]);
    if (rc == DG_OK)
        rc = capture(b, [b](hipStream_t s) { return enqueue_finish(b, s); }, &b->g_finish);
    if (rc != DG_OK) { destroy_graphs(b); return rc; }
    b->graphs_valid = true;
    return DG_OK;
}

int run(dg_batch* b, int (*fn)(dg_batch*, hipStream_t), hipGraphExec_t g, hipStream_t s) {
    if (b->use_graphs) {
        HIP_TRY(hipGraphLaunch(g, s));
        return DG_OK;
    }
    return fn(b, s);
}

// Launch groups with a member whose solve is still running (h: polled
// scalars).
unsigned running_groups(const dg_batch* b, const CgScalars* h) {
    unsigned m = 0;
    for (int i = 0; i < b->capacity; ++i)
        if (b->slots[i].used && !h[i].done) m |= 1u << group_of(b->h_inst[i].g);
    return m;
}

}  // namespace

extern "C" {

int dg_batch_create(int capacity, dg_batch** out) {
    if (!out || capacity < 1 || capacity > 4096)
        return fail(DG_E_INVAL, "capacity must be in [1, 4096]");
    *out = nullptr;
    dg_batch* b = new (std::nothrow) dg_batch;
    if (!b) return fail(DG_E_NOMEM, "host allocation failed");
    b->capacity = capacity;
    b->slots.resize(capacity);
    bool ok = hipGetDevice(&b->device) == hipSuccess &&
              hipMalloc((void**)&b->d_inst, capacity * sizeof(BatchInst)) == hipSuccess &&
              hipHostMalloc((void**)&b->h_inst, capacity * sizeof(BatchInst)) == hipSuccess &&
              hipMalloc((void**)&b->d_sc, capacity * sizeof(CgScalars)) == hipSuccess &&
              hipHostMalloc((void**)&b->h_sc, 3 * capacity * sizeof(CgScalars)) == hipSuccess &&
              hipMalloc((void**)&b->d_counts, kGroups * kListCount * sizeof(int)) == hipSuccess &&
              hipHostMalloc((void**)&b->h_counts, kGroups * kListCount * sizeof(int)) == hipSuccess &&
              hipEventCreateWithFlags(&b->ev[0], hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&b->ev[1], hipEventDisableTiming) == hipSuccess &&
              hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) == hipSuccess;
    if (ok) {
        std::memset(b->h_inst, 0, capacity * sizeof(BatchInst));
        std::memset(b->h_counts, 0, kGroups * kListCount * sizeof(int));
        ok = hipMemset(b->d_sc, 0, capacity * sizeof(CgScalars)) == hipSuccess &&
             hipMemset(b->d_counts, 0, kGroups * kListCount * sizeof(int)) == hipSuccess &&
             hipDeviceSynchronize() == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        dg_batch_destroy(b);
        return fail(DG_E_NOMEM, "batch allocation failed");
    }
    *out = b;
    return DG_OK;
}

void dg_batch_destroy(dg_batch* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    destroy_graphs(b);
    for (Slot& s : b->slots) {
        dg_workspace_destroy(s.ws);
        dg_state_destroy(s.st);
    }
    for (auto& row : b->lists)
        for (DevList& L : row)
            if (L.items) (void)hipFree(L.items);
    if (b->d_inst) (void)hipFree(b->d_inst);
    if (b->h_inst) (void)hipHostFree(b->h_inst);
    if (b->d_sc) (void)hipFree(b->d_sc);
    if (b->h_sc) (void)hipHostFree(b->h_sc);
    if (b->d_counts) (void)hipFree(b->d_counts);
    if (b->h_counts) (void)hipHostFree(b->h_counts);
    for (hipEvent_t e : b->ev) if (e) (void)hipEventDestroy(e);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

int dg_batch_attach(dg_batch* b, const dg_grid* g, double* omega, double dt,
                    double D, double t0, int* slot) {
    if (!b || !g || !omega || !slot) return fail(DG_E_INVAL, "NULL argument");
    // the fused kernels carry no Dirichlet closure; members of a batch with
    // the preconditioner step through dg_rk_step, which has it
    if ((g->geom.bcx || g->geom.bcy) && !b->fd_flags)
        return periodic_only("the fused batch steps (a batch made with dg_batch_use_precond "
                             "takes Dirichlet members)");
    if (!std::isfinite(dt) || !std::isfinite(D)) return fail(DG_E_INVAL, "dt, D must be finite");
    int i = 0;
    while (i < b->capacity && b->slots[i].used) ++i;
    if (i == b->capacity) return fail(DG_E_INVAL, "batch is full (%d slots)", b->capacity);
    Slot& sl = b->slots[i];
    int rc = dg_workspace_create(g, DG_PREC_FP64 | b->fd_flags, &sl.ws);
    if (rc != DG_OK) return rc;
    // the fused steps are never queued ahead; preconditioned members step
    // through dg_rk_step, whose queued steps keep two more psi buffers
    rc = state_create(g, t0, b->fd_flags ? 5 : 3, &sl.st);
    if (rc != DG_OK) { dg_workspace_destroy(sl.ws); sl.ws = nullptr; return rc; }
    sl.used = true;
    sl.grid = g;
    sl.omega = omega;
    sl.dt = dt;
    sl.D = D;
    BatchInst& r = b->h_inst[i];
    std::memset(&r, 0, sizeof r);
    r.g = g->geom;
    fill_batch_geometry(r);
    r.area = g->area;
    r.k = g->k64;
    r.active = 1;
    r.x = sl.ws->x;
    r.r = sl.ws->r;
    r.p0 = sl.ws->p0;
    r.p1 = sl.ws->p1;
    r.sc = b->d_sc + i;
    r.counters = sl.ws->d.counters;
    r.partials = sl.ws->d.partials;
    b->lists_dirty = true;
    *slot = i;
    return DG_OK;
}

int dg_batch_detach(dg_batch* b, int slot) {
    if (!b || slot < 0 || slot >= b->capacity || !b->slots[slot].used)
        return fail(DG_E_INVAL, "no instance in slot %d", slot);
    HIP_TRY(hipDeviceSynchronize());
    Slot& sl = b->slots[slot];
    dg_workspace_destroy(sl.ws);
    dg_state_destroy(sl.st);
    sl = Slot{};
    b->h_inst[slot].active = 0;
    b->lists_dirty = true;
    return DG_OK;
}

int dg_batch_use_precond(dg_batch* b, int ws_fd_flags) {
    if (!b) return fail(DG_E_INVAL, "NULL argument");
    if (ws_fd_flags != 0 && ws_fd_flags != DG_WS_FD &&
        ws_fd_flags != (DG_WS_FD | DG_WS_FD_PRODUCTS))
        return fail(DG_E_INVAL, "ws_fd_flags must be 0, DG_WS_FD or DG_WS_FD | DG_WS_FD_PRODUCTS");
    for (const Slot& sl : b->slots)
        if (sl.used) return fail(DG_E_INVAL, "the preconditioner is chosen before members attach");
    b->fd_flags = ws_fd_flags;
    return DG_OK;
}

int dg_batch_use_graphs(dg_batch* b, int on) {
    if (!b) return fail(DG_E_INVAL, "NULL argument");
    b->use_graphs = on != 0;
    return DG_OK;
}

// Preconditioned steps: the preconditioner's transforms and bases are per
// grid, so each member takes its step through dg_rk_step on the batch's
// stream (queued FP64-preconditioned stages, or the polled FP32-applied
// preconditioner), one member after the other: the same kernels and results
// as stand-alone steps, without the fused launches.
static int rk_step_members(dg_batch* b, const dg_cg_opts& o, int* iters_out, void* stream) {
    if (!b->fd_flags)
        return fail(DG_E_WORKSPACE, "preconditioned batch steps need dg_batch_use_precond "
                    "before the members attach");
    bool all_conv = true;
    for (int i = 0; i < b->capacity; ++i) {
        Slot& sl = b->slots[i];
        if (!sl.used) continue;
        dg_step_opts so;
        std::memset(&so, 0, sizeof so);
        so.dt = sl.dt;
        so.D = sl.D;
        so.cg = o;
        so.form = DG_FORM_ARAKAWA;
        dg_step_stats st;
        std::memset(&st, 0, sizeof st);
        const int rc = dg_rk_step(sl.grid, sl.omega, sl.st, &so, &st, sl.ws, stream);
        if (rc != DG_OK && rc != DG_E_NOCONV) return rc;
        sl.converged = rc == DG_OK;
        all_conv = all_conv && sl.converged;
        if (iters_out)
            for (int k = 0; k < 3; ++k) iters_out[3 * i + k] = st.cg_iters[k];
    }
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    if (!all_conv) return fail(DG_E_NOCONV, "a batched solve did not converge");
    return DG_OK;
}

int dg_batch_rk_step(dg_batch* b, const dg_cg_opts* opts, int* iters_out,
                     void* stream) {
    if (!b) return fail(DG_E_INVAL, "NULL argument");
    dg_cg_opts o;
    if (opts) o = *opts;
    else { o.rtol = 1e-12; o.max_iter = 100000; o.precision = DG_PREC_FP64;
           o.precond = DG_PRECOND_NONE; o.check_every = 0; }
    if (!(o.rtol > 0) || o.max_iter < 0) return fail(DG_E_INVAL, "bad CG options");
    if (o.precond == DG_PRECOND_FD) return rk_step_members(b, o, iters_out, stream);
    if (o.precision != DG_PREC_FP64 || o.precond != DG_PRECOND_NONE)
        return fail(DG_E_UNSUPPORTED, "fused batch steps run the unpreconditioned FP64 CG");
    for (const Slot& sl : b->slots)
        if (sl.used && (sl.grid->geom.bcx || sl.grid->geom.bcy))
            return periodic_only("the fused batch steps");
    hipStream_t s = (hipStream_t)stream;
    int used = 0;
    for (const Slot& sl : b->slots) used += sl.used;
    if (used == 0) return DG_OK;
    if (b->lists_dirty) {
        int rc = rebuild_lists(b, s);
        if (rc != DG_OK) return rc;
    }
    if (b->use_graphs) {
        int rc = ensure_graphs(b);
        if (rc != DG_OK) return rc;
    }
    const double ra_a[3] = {0.0, 0.75, 1.0 / 3.0};
    const double ra_b[3] = {1.0, 0.25, 2.0 / 3.0};
    bool all_conv = true;
    for (Slot& sl : b->slots) sl.converged = true;
    for (int k = 0; k < 3; ++k) {
        std::vector<int> xi(b->capacity, -1);
        std::vector<double> ts(b->capacity, 0.0);
        for (int i = 0; i < b->capacity; ++i) {
            Slot& sl = b->slots[i];
            if (!sl.used) continue;
            BatchInst& r = b->h_inst[i];
            const double t = sl.st->t;
            ts[i] = (k == 0) ? t : (k == 1 ? t + sl.dt : t + 0.5 * sl.dt);
            double* x;
            state_guess(sl.st, ts[i], &r.pa, &r.ca, &r.pb, &r.cb, &x, &xi[i]);
            r.psi = x;
            double* win[3] = {sl.omega, sl.ws->s1, sl.ws->s2};
            double* wout[3] = {sl.ws->s1, sl.ws->s2, sl.omega};
            r.w_in = win[k];
            r.w_out = wout[k];
            r.w_n = k ? sl.omega : nullptr;
            r.ra = RhsArgs{1.0, 1.0, 1.0, 1.0 / 3.0, sl.D, sl.dt, ra_a[k], ra_b[k], 0};
            r.tol2 = o.rtol * o.rtol;
            r.max_iter = o.max_iter;
        }
        HIP_TRY(hipMemcpyAsync(b->d_inst, b->h_inst, b->capacity * sizeof(BatchInst),
                               hipMemcpyHostToDevice, s));
        int rc = run(b, enqueue_setup, b->g_setup, s);
        if (rc != DG_OK) return rc;
        // CG chunks, polled one chunk behind; a group drops out once all its
        // members were seen done
        int issued = 0, round = 0, prev = -1;
        unsigned live = b->group_mask;
        for (;;) {
            for (int gi = 0; gi < kGroups; ++gi) {
                if (!(live & (1u << gi))) continue;
                if (b->use_graphs) {
                    HIP_TRY(hipGraphLaunch(b->g_chunk[gi], s));
                } else {
                    rc = enqueue_chunk(b, gi, s);
                    if (rc != DG_OK) return rc;
                }
            }
            issued += b->chunk;
            const int slot = round & 1;
            HIP_TRY(hipMemcpyAsync(b->h_sc + slot * b->capacity, b->d_sc,
                                   b->capacity * sizeof(CgScalars),
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipEventRecord(b->ev[slot], s));
            if (issued >= o.max_iter + b->chunk) {
                HIP_TRY(hipEventSynchronize(b->ev[slot]));
                break;
            }
            if (prev >= 0) {
                HIP_TRY(hipEventSynchronize(b->ev[prev]));
                live &= running_groups(b, b->h_sc + prev * b->capacity);
                if (!live) break;
            }
            prev = slot;
            ++round;
        }
        rc = run(b, enqueue_finish, b->g_finish, s);
        if (rc != DG_OK) return rc;
        CgScalars* fin = b->h_sc + 2 * b->capacity;
        HIP_TRY(hipMemcpyAsync(fin, b->d_sc, b->capacity * sizeof(CgScalars),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int i = 0; i < b->capacity; ++i) {
            Slot& sl = b->slots[i];
            if (!sl.used) continue;
            state_push(sl.st, xi[i], ts[i]);
            if (!fin[i].converged) { all_conv = false; sl.converged = false; }
            if (iters_out) iters_out[3 * i + k] = fin[i].iter;
        }
    }
    for (Slot& sl : b->slots)
        if (sl.used) sl.st->t += sl.dt;
    if (!all_conv) return fail(DG_E_NOCONV, "a batched solve did not converge");
    return DG_OK;
}

int dg_batch_slot_converged(const dg_batch* b, int slot) {
    if (!b || slot < 0 || slot >= b->capacity || !b->slots[slot].used)
        return fail(DG_E_INVAL, "no instance in slot %d", slot);
    return b->slots[slot].converged ? 1 : 0;
}

int dg_batch_copy_psi(const dg_batch* b, int slot, double* out, void* stream) {
    if (!b || slot < 0 || slot >= b->capacity || !b->slots[slot].used)
        return fail(DG_E_INVAL, "no instance in slot %d", slot);
    return dg_state_copy_psi(b->slots[slot].st, out, stream);
}

double dg_batch_time(const dg_batch* b, int slot) {
    if (!b || slot < 0 || slot >= b->capacity || !b->slots[slot].used) return 0.0;
    return b->slots[slot].st->t;
}

int dg_batch_member_bytes(const dg_grid* g, size_t* bytes) {
    if (!g || !bytes) return fail(DG_E_INVAL, "NULL argument");
    size_t w = 0;
    int rc = dg_workspace_bytes(g, DG_PREC_FP64, &w);
    if (rc != DG_OK) return rc;
    *bytes = w + 3 * g->elems * sizeof(double) + sizeof(BatchInst);
    return DG_OK;
}

}  // extern "C"
