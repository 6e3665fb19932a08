// Batched runtime of libsgweno: many solves (any dimension, level and final
// time, one precision) advance together.  A time step is the time-step kernel
// for every slot, then per dimension present one persistent launch that runs
// all three TVD-RK3 stages of the grids that are one stage box, and three
// persistent launches, one per stage, over the boxes of the other grids.  The
// box list, grouped by dimension and kind, and the ranges of it live in device
// memory, so admitting or releasing a solve is a stream-ordered copy and the
// graph stays valid.  Graphs of 1, 2, 4, ..., 2^(SGW_GRAPH_LEVELS-1) steps are
// captured, and a request for n steps launches the binary decomposition of n
// (each graph launch costs the device a gap of several microseconds, as long as
// a small stage).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sgw_api_internal.h"

struct sgw_batch {
    int max_solvers = 0;
    int precision = 0;
    uint64_t budget = 0, used = 0;
    hipStream_t stream = nullptr;
    unsigned char* scratch = nullptr;
    uint64_t scratch_bytes = 0;
    int64_t max_items = 0;
    ReqDev** reqs_d = nullptr;      // [max_solvers], null for a free slot
    WorkItem* items_d = nullptr;    // [max_items], grouped by dimension
    int* ranges_d = nullptr;        // ranges_h on the device
    int* flags_d = nullptr;         // [max_solvers]
    double* tf_d = nullptr;         // [max_solvers] final times of new slots (NaN: unchanged)
    int* flags_pinned = nullptr;
    hipEvent_t ev_order = nullptr;  // orders a released solver's own stream after the batch's steps
    hipEvent_t ev_admit = nullptr;  // orders the batch stream after an admitted solver's own work
    hipEvent_t ev_poll = nullptr;   // behind the copy of the completion flags
    bool poll_inflight = false;
    std::vector<uint64_t> slot_gen;   // bumped by every admission and release of the slot
    std::vector<uint64_t> poll_gen;   // slot_gen when the flags in flight were gathered
    std::vector<sgw_solver*> slots;
    int free_hint = 0;              // no free slot below this index
    int64_t items_admitted = 0;     // boxes of the admitted solves
    std::vector<uint64_t> slot_bytes;
    std::vector<ReqDev*> reqs_h;
    std::vector<double> tf_h;
    bool tf_pending = false;
    bool queued = false;            // step launches may still be in flight on the stream
    std::vector<WorkItem> items_h;
    int nitems_h = 0;
    // (offset, count) in the box list, [kind][dimension - 1]: kind 0 the grids that are one
    // box (three-stage launch), 1 the boxes of the other grids, 2 both (contiguous)
    int ranges_h[3][4][2] = {};
    bool dirty = true;
    size_t lds[2][4] = {};          // LDS of the captured launches, [kind][dimension - 1] (0: not captured)
    int blocks[2][4] = {};
    // the 3D solvers of a batch share one sweep form: line sweeps (lines3) or stage boxes; the
    // captured graphs were built for cap_lines3
    bool lines3 = false, cap_lines3 = false;
    int blocks_per_cu = 0;          // cap on resident stage workgroups per CU (0: occupancy)
    hipStream_t cap = nullptr;
    hipGraph_t graph[6] = {};           // graph[j]: 2^j steps
    hipGraphExec_t exec[6] = {};
};

#define SGW_GRAPH_LEVELS 6

static uint64_t a256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

extern "C" uint64_t sgw_batch_scratch_bytes(int32_t max_solvers, int64_t max_items)
{
    if (max_solvers < 1 || max_items < 1) return 0;
    return a256(sizeof(ReqDev*) * (uint64_t)max_solvers) + a256(sizeof(WorkItem) * (uint64_t)max_items) + 256 +
           a256(sizeof(int) * (uint64_t)max_solvers) + a256(sizeof(double) * (uint64_t)max_solvers);
}

extern "C" sgw_status sgw_batch_create(int32_t max_solvers, int32_t precision, uint64_t hbm_budget, void* hip_stream,
                                       void* scratch_dev, uint64_t scratch_bytes, sgw_batch_t** out)
{
    if (!out || !scratch_dev) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (max_solvers < 1 || max_solvers > 65536) return sgw_fail(SGW_ERR_INVALID_ARG, "max_solvers %d", max_solvers);
    if (precision != SGW_FP64 && precision != SGW_FP32_SWEEP)
        return sgw_fail(SGW_ERR_INVALID_ARG, "unknown precision %d", precision);
    if ((uintptr_t)scratch_dev & 255) return sgw_fail(SGW_ERR_INVALID_ARG, "scratch must be 256-byte aligned");
    const uint64_t fixed = sgw_batch_scratch_bytes(max_solvers, 1) - a256(sizeof(WorkItem));
    if (scratch_bytes < fixed + a256(sizeof(WorkItem))) return sgw_fail(SGW_ERR_OUT_OF_MEMORY, "batch scratch too small");
    sgw_batch* b = new sgw_batch();
    b->max_solvers = max_solvers;
    b->precision = precision;
    b->budget = hbm_budget;
    b->stream = (hipStream_t)hip_stream;
    b->scratch = (unsigned char*)scratch_dev;
    b->scratch_bytes = scratch_bytes;
    b->max_items = (int64_t)((scratch_bytes - fixed) / sizeof(WorkItem));
    if (b->max_items > (1ll << 30)) b->max_items = 1ll << 30;
    uint64_t off = 0;
    b->reqs_d = (ReqDev**)(b->scratch + off);
    off += a256(sizeof(ReqDev*) * (uint64_t)max_solvers);
    b->ranges_d = (int*)(b->scratch + off);
    off += 256;
    b->flags_d = (int*)(b->scratch + off);
    off += a256(sizeof(int) * (uint64_t)max_solvers);
    b->tf_d = (double*)(b->scratch + off);
    off += a256(sizeof(double) * (uint64_t)max_solvers);
    b->items_d = (WorkItem*)(b->scratch + off);
    b->slots.assign(max_solvers, nullptr);
    b->slot_gen.assign(max_solvers, 0);
    b->poll_gen.assign(max_solvers, 0);
    b->slot_bytes.assign(max_solvers, 0);
    b->reqs_h.assign(max_solvers, nullptr);
    b->tf_h.assign(max_solvers, NAN);
    hipError_t e = hipHostMalloc((void**)&b->flags_pinned, sizeof(int) * max_solvers, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_order, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_admit, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_poll, hipEventDisableTiming);
    if (e != hipSuccess) {
        sgw_batch_free(b);
        return sgw_hip_fail(e, "batch set-up");
    }
    *out = b;
    return SGW_OK;
}

static void batch_drop_graph(sgw_batch* b)
{
    for (int j = 0; j < SGW_GRAPH_LEVELS; j++) {
        if (b->exec[j]) (void)hipGraphExecDestroy(b->exec[j]);
        if (b->graph[j]) (void)hipGraphDestroy(b->graph[j]);
        b->exec[j] = nullptr;
        b->graph[j] = nullptr;
    }
    if (b->cap) (void)hipStreamDestroy(b->cap);
    b->cap = nullptr;
}

extern "C" void sgw_batch_free(sgw_batch_t* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    batch_drop_graph(b);
    for (auto* s : b->slots)
        if (s) s->batch_slot = -1;
    if (b->flags_pinned) (void)hipHostFree(b->flags_pinned);
    if (b->ev_order) (void)hipEventDestroy(b->ev_order);
    if (b->ev_admit) (void)hipEventDestroy(b->ev_admit);
    if (b->ev_poll) (void)hipEventDestroy(b->ev_poll);
    delete b;
}

static uint64_t solver_bytes(const sgw_solver* s)
{
    return s->plan->state_bytes + s->plan->scratch_bytes + (uint64_t)s->plan->fine_nodes * sizeof(double);
}

// The stage launches of one step (stage < 0): for every captured dimension, the three-stage
// launch over its one-box grids, then stage by stage the launches over the boxes of the
// other grids.  stage 0..2: that stage alone over all boxes (the split kernel, every box);
// SGW_STAGE_FUSED: the launches of a step over the current lists, captured or not.
static hipError_t enqueue_stages(sgw_batch* b, int stage, hipStream_t st)
{
    hipError_t e = hipSuccess;
    const bool step = stage < 0 || stage == SGW_STAGE_FUSED;
    if (!step) {
        for (int d = 0; d < 4 && e == hipSuccess; d++) {
            if (!b->ranges_h[2][d][1]) continue;
            const size_t l = b->lds[0][d] > b->lds[1][d] ? b->lds[0][d] : b->lds[1][d];
            e = launch_stage_range(b->items_d, b->ranges_d + (2 * 4 + d) * 2,
                                   stage_grid(b->precision, d + 1, l, b->blocks_per_cu), stage, b->precision, d + 1, l,
                                   st, d == 3 || (d == 2 && b->lines3));
        }
        return e;
    }
    // a captured graph keeps every launch it was built with; a direct call skips empty ranges
    const bool all = stage < 0;
    for (int d = 0; d < 4 && e == hipSuccess; d++)
        if (b->lds[0][d] && (all || b->ranges_h[0][d][1]))
            e = launch_stage_range(b->items_d, b->ranges_d + d * 2, b->blocks[0][d], SGW_STAGE_FUSED, b->precision,
                                   d + 1, b->lds[0][d], st);
    for (int s = 0; s < 3 && e == hipSuccess; s++)
        for (int d = 0; d < 4 && e == hipSuccess; d++)
            if (b->lds[1][d] && (all || b->ranges_h[1][d][1]))
                e = launch_stage_range(b->items_d, b->ranges_d + (4 + d) * 2, b->blocks[1][d], s, b->precision, d + 1,
                                       b->lds[1][d], st, d == 3 || (d == 2 && b->lines3));
    return e;
}

// Re-upload the box list and the slot table; recapture the step graphs only when
// a solve of a kind of launch (dimension; one-box grids or not) not yet captured
// arrives, or an admitted grid needs more LDS than the captured launch provides.
// Captured launches stay in the graph (an empty range costs one launch whose
// workgroups exit).
static sgw_status batch_sync(sgw_batch* b)
{
    if (!b->dirty) return SGW_OK;
    b->items_h.clear();
    size_t lds[2][4] = {};
    for (int d = 1; d <= 4; d++) {
        const size_t d_begin = b->items_h.size();
        for (int kind = 0; kind < 2; kind++) {
            b->ranges_h[kind][d - 1][0] = (int)b->items_h.size();
            for (int i = 0; i < b->max_solvers; i++) {
                sgw_solver* s = b->slots[i];
                if (!s || s->plan->pb.dim != d) continue;
                const sgw_plan* p = s->plan;
                // a solver's list holds its one-box grids first
                const size_t lo = kind == 0 ? 0 : (size_t)p->nitems_whole;
                const size_t hi = kind == 0 ? (size_t)p->nitems_whole : (size_t)p->nitems;
                if (hi == lo) continue;
                if ((int64_t)(b->items_h.size() + (hi - lo)) > b->max_items)
                    return sgw_fail(SGW_ERR_OUT_OF_MEMORY, "batch box list full");
                b->items_h.insert(b->items_h.end(), s->items_h.begin() + lo, s->items_h.begin() + hi);
                const size_t l = kind == 0 ? p->lds_whole : p->lds_boxed;
                lds[kind][d - 1] = l > lds[kind][d - 1] ? l : lds[kind][d - 1];
            }
            b->ranges_h[kind][d - 1][1] = (int)b->items_h.size() - b->ranges_h[kind][d - 1][0];
        }
        b->ranges_h[2][d - 1][0] = (int)d_begin;
        b->ranges_h[2][d - 1][1] = (int)(b->items_h.size() - d_begin);
    }
    b->nitems_h = (int)b->items_h.size();
    // the lists go through a pinned staging buffer: the uploads are stream-ordered
    // and the host does not wait for the device
    const size_t n_items = sizeof(WorkItem) * b->items_h.size(), n_ranges = sizeof(b->ranges_h);
    const size_t n_reqs = sizeof(ReqDev*) * b->max_solvers, n_tf = sizeof(double) * b->max_solvers;
    Staging stg(n_items + n_ranges + n_reqs + n_tf);
    hipError_t e = stg.err;
    if (e == hipSuccess) {
        unsigned char* h = stg.host;
        if (n_items) std::memcpy(h, b->items_h.data(), n_items);
        std::memcpy(h + n_items, b->ranges_h, n_ranges);
        std::memcpy(h + n_items + n_ranges, b->reqs_h.data(), n_reqs);
        std::memcpy(h + n_items + n_ranges + n_reqs, b->tf_h.data(), n_tf);
        e = stg.upload(0, b->items_d, n_items, b->stream);
    }
    if (e == hipSuccess) e = stg.upload(n_items, b->ranges_d, n_ranges, b->stream);
    if (e == hipSuccess) e = stg.upload(n_items + n_ranges, b->reqs_d, n_reqs, b->stream);
    if (e == hipSuccess && b->tf_pending) {
        e = stg.upload(n_items + n_ranges + n_reqs, b->tf_d, n_tf, b->stream);
        if (e == hipSuccess) e = launch_req_set_final_many(b->reqs_d, b->tf_d, b->max_solvers, b->stream);
    }
    if (e != hipSuccess) return sgw_hip_fail(e, "upload batch lists");
    if (b->tf_pending) {
        for (double& t : b->tf_h) t = NAN;
        b->tf_pending = false;
    }
    bool recapture = false;
    for (int j = 0; j < SGW_GRAPH_LEVELS; j++) recapture |= !b->exec[j];
    for (int i = 0; i < b->max_solvers; i++)
        if (b->slots[i] && b->slots[i]->plan->pb.dim == 3) {
            b->lines3 = b->slots[i]->plan->line_mode;
            break;
        }
    recapture |= b->lines3 != b->cap_lines3;
    for (int k = 0; k < 2; k++)
        for (int d = 0; d < 4; d++) recapture |= lds[k][d] > b->lds[k][d];
    if (recapture) {
        // queued launches of the old graphs may still run: wait before they are destroyed
        if (b->queued) {
            e = hipStreamSynchronize(b->stream);
            if (e != hipSuccess) return sgw_hip_fail(e, "synchronise batch");
            b->queued = false;
        }
        batch_drop_graph(b);
        for (int k = 0; k < 2; k++)
            for (int d = 0; d < 4; d++) {
                b->lds[k][d] = lds[k][d] > b->lds[k][d] ? lds[k][d] : b->lds[k][d];
                b->blocks[k][d] =
                    b->lds[k][d] ? stage_grid(b->precision, d + 1, b->lds[k][d], b->blocks_per_cu, k == 0) : 0;
            }
        b->cap_lines3 = b->lines3;
        e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
        if (e != hipSuccess) return sgw_hip_fail(e, "capture stream");
        for (int which = 0; which < SGW_GRAPH_LEVELS; which++) {
            const int nsteps = 1 << which;
            e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return sgw_hip_fail(e, "begin capture");
            hipError_t el = hipSuccess;
            for (int step = 0; step < nsteps && el == hipSuccess; step++) {
                el = launch_dt(b->reqs_d, b->max_solvers, b->cap);
                if (el == hipSuccess) el = enqueue_stages(b, -1, b->cap);
            }
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(b->cap, &g);
            if (el != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return sgw_hip_fail(el, "capture batch step");
            }
            if (e != hipSuccess) return sgw_hip_fail(e, "end capture");
            hipGraphExec_t x = nullptr;
            e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
            b->graph[which] = g;
            if (e != hipSuccess) return sgw_hip_fail(e, "instantiate batch graph");
            b->exec[which] = x;
        }
    }
    b->dirty = false;
    return SGW_OK;
}

// The batch stream waits (an event, no host wait) for the work already enqueued on a
// solver's own stream, such as its restriction.
static sgw_status order_after_solver_stream(sgw_batch_t* b, hipStream_t ss)
{
    if (ss == b->stream) return SGW_OK;
    hipError_t e = hipEventRecord(b->ev_admit, ss);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_admit, 0);
    if (e != hipSuccess) return sgw_hip_fail(e, "order batch after solver stream");
    return SGW_OK;
}

// ordered: the caller has already ordered the batch stream after the solver's stream
static sgw_status admit_one(sgw_batch_t* b, sgw_solver_t* s, double t_final, int32_t* slot, bool ordered)
{
    if (!b || !s || !slot) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    if (!s->restricted) return sgw_fail(SGW_ERR_STATE, "admit before restrict");
    if (s->batch_slot >= 0) return sgw_fail(SGW_ERR_STATE, "solver already in a batch");
    if (s->plan->cfg.precision != b->precision) return sgw_fail(SGW_ERR_INVALID_ARG, "precision differs from batch");
    // a batch runs its 4D grids as line sweeps
    if (s->plan->pb.dim == 4 && !s->plan->line_mode)
        return sgw_fail(SGW_ERR_UNSUPPORTED, "4D solvers with manual stage boxes run alone, not in a batch");
    // the batch launches carry no density pass
    if (s->plan->relax || s->plan->zmask || s->plan->vm)
        return sgw_fail(SGW_ERR_UNSUPPORTED,
                        "zero-boundary, relaxation and Vlasov-Maxwell solvers run alone, not in a batch");
    // its 3D solvers share one sweep form (line sweeps, or stage boxes with sweep_form 2)
    if (s->plan->pb.dim == 3)
        for (int i = 0; i < b->max_solvers; i++)
            if (b->slots[i] && b->slots[i]->plan->pb.dim == 3 && b->slots[i]->plan->line_mode != s->plan->line_mode)
                return sgw_fail(SGW_ERR_UNSUPPORTED,
                                "3D solvers of one batch share their sweep form (line sweeps or stage boxes)");
    if (!(t_final >= 0.0)) return sgw_fail(SGW_ERR_INVALID_ARG, "bad final time");
    const uint64_t need = solver_bytes(s);
    if (b->used + need > b->budget)
        return sgw_fail(SGW_ERR_OUT_OF_MEMORY, "footprint %llu exceeds remaining budget %llu",
                        (unsigned long long)need, (unsigned long long)(b->budget - b->used));
    int free_slot = -1;
    for (int i = b->free_hint; i < b->max_solvers; i++)
        if (!b->slots[i]) {
            free_slot = i;
            break;
        }
    if (free_slot < 0) return sgw_fail(SGW_ERR_OUT_OF_MEMORY, "no free slot");
    b->free_hint = free_slot;
    if (b->items_admitted + (int64_t)s->items_h.size() > b->max_items)
        return sgw_fail(SGW_ERR_OUT_OF_MEMORY, "box list full");
    // the solve's own work (restriction) is ordered before the batch's
    if (!ordered) {
        const sgw_status rc = order_after_solver_stream(b, s->stream);
        if (rc != SGW_OK) return rc;
    }
    // the final time reaches the device with the next upload of the slot table
    b->tf_h[free_slot] = t_final;
    b->tf_pending = true;
    b->slots[free_slot] = s;
    b->slot_gen[free_slot]++;
    b->items_admitted += (int64_t)s->items_h.size();
    b->slot_bytes[free_slot] = need;
    b->reqs_h[free_slot] = s->req_d;
    b->used += need;
    s->batch_slot = free_slot;
    b->dirty = true;
    *slot = free_slot;
    return SGW_OK;
}

extern "C" sgw_status sgw_batch_admit(sgw_batch_t* b, sgw_solver_t* s, double t_final, int32_t* slot)
{
    return admit_one(b, s, t_final, slot, false);
}

extern "C" sgw_status sgw_batch_step(sgw_batch_t* b, int32_t nsteps)
{
    if (!b) return sgw_fail(SGW_ERR_INVALID_ARG, "null batch");
    if (nsteps < 0) return sgw_fail(SGW_ERR_INVALID_ARG, "negative step count");
    sgw_status rc = batch_sync(b);
    if (rc != SGW_OK) return rc;
    if (!b->nitems_h) return SGW_OK;
    for (int left = nsteps; left > 0;) {
        int j = SGW_GRAPH_LEVELS - 1;
        while ((1 << j) > left) j--;
        b->queued = true;
        hipError_t e = hipGraphLaunch(b->exec[j], b->stream);
        if (e != hipSuccess) return sgw_hip_fail(e, "batch graph launch");
        left -= 1 << j;
    }
    return SGW_OK;
}

extern "C" sgw_status sgw_batch_poll_begin(sgw_batch_t* b)
{
    if (!b) return sgw_fail(SGW_ERR_INVALID_ARG, "null batch");
    if (b->poll_inflight) return sgw_fail(SGW_ERR_STATE, "a poll is already in flight");
    sgw_status rc = batch_sync(b);
    if (rc != SGW_OK) return rc;
    hipError_t e = launch_gather_done(b->reqs_d, b->max_solvers, b->flags_d, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->flags_pinned, b->flags_d, sizeof(int) * b->max_solvers, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->ev_poll, b->stream);
    if (e != hipSuccess) return sgw_hip_fail(e, "poll batch");
    b->poll_gen = b->slot_gen;
    b->poll_inflight = true;
    return SGW_OK;
}

extern "C" sgw_status sgw_batch_poll_end(sgw_batch_t* b, int32_t* done_slots, int32_t* n_done)
{
    if (!b || !done_slots || !n_done) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    if (!b->poll_inflight) return sgw_fail(SGW_ERR_STATE, "no poll in flight");
    b->poll_inflight = false;
    hipError_t e = hipEventSynchronize(b->ev_poll);
    if (e != hipSuccess) return sgw_hip_fail(e, "poll batch");
    int n = 0;
    bool bad = false;
    for (int i = 0; i < b->max_solvers; i++) {
        // a slot released or refilled since the flags were gathered is not reported (also
        // when the same solver was admitted again)
        if (!b->slots[i] || b->slot_gen[i] != b->poll_gen[i]) continue;
        if (b->flags_pinned[i] & 1) done_slots[n++] = i;
        bad |= (b->flags_pinned[i] & 2) != 0;
    }
    *n_done = n;
    if (bad) return sgw_fail(SGW_ERR_NONFINITE, "a solve in the batch hit a non-finite wave speed");
    return SGW_OK;
}

extern "C" sgw_status sgw_batch_poll(sgw_batch_t* b, int32_t* done_slots, int32_t* n_done)
{
    if (!b || !done_slots || !n_done) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    sgw_status rc = sgw_batch_poll_begin(b);
    if (rc != SGW_OK) return rc;
    rc = sgw_batch_poll_end(b, done_slots, n_done);
    // nothing is queued behind the flags: every step launched so far has run
    if (rc == SGW_OK || rc == SGW_ERR_NONFINITE) b->queued = false;
    return rc;
}

extern "C" sgw_status sgw_batch_launch_stage(sgw_batch_t* b, int32_t stage, int32_t reps)
{
    if (!b) return sgw_fail(SGW_ERR_INVALID_ARG, "null batch");
    if (stage < 0 || stage > SGW_STAGE_FUSED || reps < 0)
        return sgw_fail(SGW_ERR_INVALID_ARG, "stage %d reps %d", stage, reps);
    sgw_status rc = batch_sync(b);
    if (rc != SGW_OK) return rc;
    for (int i = 0; i < reps; i++) {
        b->queued = true;
        hipError_t e = enqueue_stages(b, stage, b->stream);
        if (e != hipSuccess) return sgw_hip_fail(e, "stage launch");
    }
    return SGW_OK;
}

extern "C" sgw_status sgw_batch_info(const sgw_batch_t* b, int32_t* active, int64_t* boxes, int64_t* nodes)
{
    if (!b) return sgw_fail(SGW_ERR_INVALID_ARG, "null batch");
    int n = 0;
    int64_t bx = 0, nd = 0;
    for (auto* s : b->slots)
        if (s) {
            n++;
            bx += (int64_t)s->items_h.size();
            nd += s->plan->total_nodes;
        }
    if (active) *active = n;
    if (boxes) *boxes = bx;
    if (nodes) *nodes = nd;
    return SGW_OK;
}

// Frees a slot whose solver's stream the caller has already ordered after the queued steps.
static void release_slot(sgw_batch_t* b, int32_t slot)
{
    sgw_solver* s = b->slots[slot];
    s->batch_slot = -1;
    b->items_admitted -= (int64_t)s->items_h.size();
    if (slot < b->free_hint) b->free_hint = slot;
    b->tf_h[slot] = NAN;
    b->used -= b->slot_bytes[slot];
    b->slots[slot] = nullptr;
    b->slot_gen[slot]++;
    b->slot_bytes[slot] = 0;
    b->reqs_h[slot] = nullptr;
    b->dirty = true;
}

extern "C" sgw_status sgw_batch_release(sgw_batch_t* b, int32_t slot)
{
    if (!b) return sgw_fail(SGW_ERR_INVALID_ARG, "null batch");
    if (slot < 0 || slot >= b->max_solvers || !b->slots[slot]) return sgw_fail(SGW_ERR_INVALID_ARG, "bad slot %d", slot);
    // queued steps may still work on the solve: its own stream waits for them
    sgw_solver* s = b->slots[slot];
    if (b->queued && s->stream != b->stream) {
        hipError_t e = hipEventRecord(b->ev_order, b->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(s->stream, b->ev_order, 0);
        if (e != hipSuccess) return sgw_hip_fail(e, "order solver stream after batch");
    }
    release_slot(b, slot);
    return SGW_OK;
}

extern "C" sgw_status sgw_batch_set_blocks_per_cu(sgw_batch_t* b, int32_t blocks_per_cu)
{
    if (!b) return sgw_fail(SGW_ERR_INVALID_ARG, "null batch");
    if (blocks_per_cu < 0 || blocks_per_cu > 64)
        return sgw_fail(SGW_ERR_INVALID_ARG, "blocks_per_cu %d outside 0..64", blocks_per_cu);
    if (blocks_per_cu == b->blocks_per_cu) return SGW_OK;
    // queued launches of the old graph may still run: wait before it is destroyed
    if (b->queued) {
        hipError_t e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return sgw_hip_fail(e, "synchronise batch");
        b->queued = false;
    }
    batch_drop_graph(b);
    for (int k = 0; k < 2; k++)
        for (int d = 0; d < 4; d++) b->lds[k][d] = 0;
    b->blocks_per_cu = blocks_per_cu;
    b->dirty = true;
    return SGW_OK;
}

extern "C" sgw_status sgw_batch_admit_many(sgw_batch_t* b, sgw_solver_t* const* solvers, int32_t n,
                                           const double* t_final, int32_t* slots, int32_t* n_admitted)
{
    if (!b || !solvers || !t_final || !slots || !n_admitted || n < 0)
        return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    *n_admitted = 0;
    // one ordering per distinct solver stream, not one per solver
    std::vector<hipStream_t> ordered;
    for (int i = 0; i < n; i++) {
        if (!solvers[i]) return sgw_fail(SGW_ERR_INVALID_ARG, "null solver %d", i);
        hipStream_t ss = solvers[i]->stream;
        if (std::find(ordered.begin(), ordered.end(), ss) != ordered.end()) continue;
        const sgw_status rc = order_after_solver_stream(b, ss);
        if (rc != SGW_OK) return rc;
        ordered.push_back(ss);
    }
    for (int i = 0; i < n; i++) {
        const sgw_status rc = admit_one(b, solvers[i], t_final[i], slots + i, true);
        if (rc != SGW_OK) return rc;
        *n_admitted = i + 1;
    }
    return SGW_OK;
}

extern "C" sgw_status sgw_batch_release_many(sgw_batch_t* b, const int32_t* slots, int32_t n)
{
    if (!b || (!slots && n > 0) || n < 0) return sgw_fail(SGW_ERR_INVALID_ARG, "null argument");
    std::vector<char> seen(b->max_solvers, 0);
    for (int i = 0; i < n; i++) {
        if (slots[i] < 0 || slots[i] >= b->max_solvers || !b->slots[slots[i]])
            return sgw_fail(SGW_ERR_INVALID_ARG, "bad slot %d", slots[i]);
        if (seen[slots[i]]++) return sgw_fail(SGW_ERR_INVALID_ARG, "slot %d listed twice", slots[i]);
    }
    // one event after the queued steps, and one wait per distinct solver stream
    if (b->queued) {
        std::vector<hipStream_t> waited;
        bool recorded = false;
        for (int i = 0; i < n; i++) {
            hipStream_t ss = b->slots[slots[i]]->stream;
            if (ss == b->stream || std::find(waited.begin(), waited.end(), ss) != waited.end()) continue;
            hipError_t e = hipSuccess;
            if (!recorded) e = hipEventRecord(b->ev_order, b->stream);
            recorded = true;
            if (e == hipSuccess) e = hipStreamWaitEvent(ss, b->ev_order, 0);
            if (e != hipSuccess) return sgw_hip_fail(e, "order solver stream after batch");
            waited.push_back(ss);
        }
    }
    for (int i = 0; i < n; i++) release_slot(b, slots[i]);
    return SGW_OK;
}
