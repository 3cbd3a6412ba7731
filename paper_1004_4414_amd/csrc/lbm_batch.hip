// Batched stepping of many lattices with one graph launch, and the tile /
// kernel autotuner.
//
// A batch captures `k` time steps of every member into one HIP graph; a
// replay advances every member by k steps with one launch.  Small members
// that share precision and collision model, use the two-pass sweep and have
// no walls are captured as shared launches: every stage of a step is one
// kernel launch over all of them, each block finding its member from block
// maps in device memory and running the same body as the single-lattice
// kernel.  The other members (large ones, a lone one of the shared kind,
// those of another kind) are captured with their own launches, each on a
// stream of its own forked from and joined into the capture stream
// (independent branches beside the shared launches).  Either way a member's
// result is bitwise the same alone and in a batch.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "lbm_handle.h"

struct lb_batch {
    std::vector<lb_handle *> m;
    std::vector<hipStream_t> branch;
    std::vector<hipEvent_t> ev_member;
    hipStream_t stream = nullptr;  // the caller's stream; replays are ordered on it
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev_done = nullptr;
    int k = 2;
    bool shared = false;            // one launch per stage for all members
    std::vector<int> cur0;          // the members' buffer parity the graph was captured with
    void *tables = nullptr;         // device member tables and block maps (shared launches)
    std::string err;
};

namespace {

// message of the last failed lb_batch_create on this thread (lb_batch_last_error(NULL))
thread_local std::string g_batch_create_error = "null batch";

int bfail(lb_batch *b, int code, const std::string &msg) {
    if (b) b->err = msg;
    else g_batch_create_error = msg;
    return code;
}

void release(lb_batch *b) {
    for (lb_handle *h : b->m) h->in_batch = false;
    if (b->tables) (void)hipFree(b->tables);
    b->tables = nullptr;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (hipStream_t s : b->branch) (void)hipStreamDestroy(s);
    for (hipEvent_t e : b->ev_member) (void)hipEventDestroy(e);
    if (b->ev_done) (void)hipEventDestroy(b->ev_done);
    b->exec = nullptr;
    b->graph = nullptr;
    b->branch.clear();
    b->ev_member.clear();
    b->ev_done = nullptr;
}

#define BATCH_CHECK(expr) LB_HIP_CHECK(expr)

// Small members that share precision and collision model, use the two-pass
// sweep and have no walls are advanced by shared launches: the member tables
// (both step parities) and the block maps go to the device once, and every
// stage of a step is one launch over all of them.  A member of SHARED_MAX_SITES
// sites or more fills the GPU with its own launches, which take their
// parameters from the kernel arguments: it keeps them, on a branch, as does
// a lone member of the shared kind.
constexpr long long SHARED_MAX_SITES = 1LL << 21;

std::vector<int> shared_members(const std::vector<lb_handle *> &m) {
    std::vector<int> sh;
    for (int i = 0; i < (int)m.size(); ++i) {
        const lb_handle *h = m[i];
        if (h->kernel != LB_KERNEL_TWOPASS || h->prm.wall_axis >= 0 || h->N >= SHARED_MAX_SITES) continue;
        if (!sh.empty()) {
            const lb_handle *h0 = m[sh[0]];
            if (h->prm.precision != h0->prm.precision || h->prm.velocity_mode != h0->prm.velocity_mode ||
                h->prm.eq_order != h0->prm.eq_order)
                continue;
        }
        sh.push_back(i);
    }
    if (sh.size() < 2) sh.clear();
    return sh;
}

void build_shared(lb_batch *b, const std::vector<lb_handle *> &ms, lbm::BatchLaunch &L) {
    using namespace lbm;
    const int nm = (int)ms.size();
    std::vector<BatchMember> tab(2 * (size_t)nm);
    std::vector<int32_t> start((size_t)BM_COUNT * (nm + 1), 0);
    for (int i = 0; i < nm; ++i) {
        lb_handle *h = ms[i];
        const bool cells = h->dpart.pgx > 0 && h->np >= PAIR_CELLS_MIN_SPHERES;
        const int np = h->np, np256 = (h->np + BLOCK - 1) / BLOCK;
        const int cnt[BM_COUNT] = {(int)((h->N + BLOCK - 1) / BLOCK), np, np256, cells ? np : 0,
                                   cells ? np256 : 0, cells && np ? 1 : 0, cells ? 0 : np};
        for (int k = 0; k < BM_COUNT; ++k) start[(size_t)k * (nm + 1) + i + 1] = start[(size_t)k * (nm + 1) + i] + cnt[k];
        for (int par = 0; par < 2; ++par) {
            BatchMember &M = tab[(size_t)par * nm + i];
            const int c = h->cur ^ par;
            M.P = h->dp;
            M.D = h->dpart;
            // a batch writes every bounced population from the link kernel
            M.P.link_write = 1;
            M.P.redirect = 0;
            M.D.track_flags = 0;
            M.fin = h->f[c];
            M.fout = h->f[1 - c];
            M.rho = h->rho;
            M.psi = h->psi;
            M.fsc = h->fsc;
            M.info = h->info;
            M.owner = h->owner;
            M.stage = h->stage;
            M.partial = h->partial;
            M.dstate = h->dstate;
            M.rows = h->prm.nx % (int)VB == 0 ? 1 : 0;
            M.cells = cells ? 1 : 0;
        }
    }
    const size_t tb = sizeof(BatchMember) * tab.size(), sb = sizeof(int32_t) * start.size();
    BATCH_CHECK(hipMalloc(&b->tables, tb + sb));
    BATCH_CHECK(hipMemcpy(b->tables, tab.data(), tb, hipMemcpyHostToDevice));
    BATCH_CHECK(hipMemcpy((char *)b->tables + tb, start.data(), sb, hipMemcpyHostToDevice));
    const BatchMember *dt = (const BatchMember *)b->tables;
    const int32_t *ds = (const int32_t *)((char *)b->tables + tb);
    for (int par = 0; par < 2; ++par) L.plan[par] = BatchPlan{dt + (size_t)par * nm, ds, nm};
    for (int k = 0; k < BM_COUNT; ++k) L.total[k] = start[(size_t)k * (nm + 1) + nm];
    L.nm = nm;
    L.fin_stride = 1;
    for (int i = 0; i < nm; ++i)
        L.fin_stride = std::max(L.fin_stride, fin_blocks((start[i + 1] - start[i]) * (int)(BLOCK / 64)));
    L.any_rows = L.any_flat = 0;
    for (int i = 0; i < nm; ++i) {
        if (ms[i]->prm.nx % (int)VB == 0) L.any_rows = 1;
        else L.any_flat = 1;
    }
    L.prm = ms[0]->prm;
}

}  // namespace

extern "C" {

int lb_batch_create(lb_handle **members, int32_t n, int32_t steps_per_launch, void *hip_stream, lb_batch **out) {
    if (!out) return bfail(nullptr, LB_EINVAL, "null output pointer");
    *out = nullptr;
    if (n < 1 || !members) return bfail(nullptr, LB_EINVAL, "no members");
    if (steps_per_launch < 2 || steps_per_launch % 2)
        return bfail(nullptr, LB_EINVAL, "steps_per_launch must be even and >= 2");
    for (int i = 0; i < n; ++i) {
        if (!members[i]) return bfail(nullptr, LB_EINVAL, "null member " + std::to_string(i));
        if (members[i]->in_batch) return bfail(nullptr, LB_EINVAL, "member " + std::to_string(i) + " is in a batch");
        if (members[i]->timing) return bfail(nullptr, LB_EINVAL, "member " + std::to_string(i) + " records timing");
        for (int j = 0; j < i; ++j)
            if (members[j] == members[i]) return bfail(nullptr, LB_EINVAL, "member " + std::to_string(i) + " repeated");
    }
    lb_batch *b = new lb_batch;
    b->m.assign(members, members + n);
    b->k = steps_per_launch;
    b->stream = (hipStream_t)hip_stream;
    std::vector<hipStream_t> saved(n);
    hipStream_t cs = nullptr;
    std::vector<hipEvent_t> joins;
    hipEvent_t fork = nullptr;
    try {
        for (lb_handle *h : b->m) {
            lbm::settle_bounces(h);  // the graph's first sweep pulls plainly
            lbm::settle_lists(h);    // and its first virtual-fluid fill reads the lists
            h->flags_tracked = false;
            BATCH_CHECK(hipStreamSynchronize(h->stream));
        }
        b->branch.resize(n);
        b->ev_member.resize(n);
        for (int i = 0; i < n; ++i) {
            BATCH_CHECK(hipStreamCreateWithFlags(&b->branch[i], hipStreamNonBlocking));
            BATCH_CHECK(hipEventCreateWithFlags(&b->ev_member[i], hipEventDisableTiming));
        }
        BATCH_CHECK(hipEventCreateWithFlags(&b->ev_done, hipEventDisableTiming));
        BATCH_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        BATCH_CHECK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        joins.resize(n, nullptr);
        for (int i = 0; i < n; ++i) BATCH_CHECK(hipEventCreateWithFlags(&joins[i], hipEventDisableTiming));
        const std::vector<int> sh = shared_members(b->m);
        std::vector<char> in_shared(n, 0);
        std::vector<lb_handle *> shm;
        for (int i : sh) {
            in_shared[i] = 1;
            shm.push_back(b->m[i]);
        }
        b->shared = !shm.empty();
        lbm::BatchLaunch L{};
        if (b->shared) build_shared(b, shm, L);
        BATCH_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        BATCH_CHECK(hipEventRecord(fork, cs));
        // the branches of the members with launches of their own ...
        for (int i = 0; i < n; ++i) {
            if (in_shared[i]) continue;
            lb_handle *h = b->m[i];
            BATCH_CHECK(hipStreamWaitEvent(b->branch[i], fork, 0));
            saved[i] = h->stream;
            h->stream = b->branch[i];
            for (int s = 0; s < b->k; ++s) lbm::one_step(h);
            h->stream = saved[i];
            h->step -= b->k;  // the capture only recorded the steps
            BATCH_CHECK(hipEventRecord(joins[i], b->branch[i]));
        }
        // ... beside the shared launches of the others
        if (b->shared)
            for (int s = 0; s < b->k; ++s) {
                lbm::launch_batch_fluid(L, s & 1, cs);
                lbm::launch_batch_particles(L, s & 1, cs);
            }
        for (int i = 0; i < n; ++i)
            if (!in_shared[i]) BATCH_CHECK(hipStreamWaitEvent(cs, joins[i], 0));
        BATCH_CHECK(hipStreamEndCapture(cs, &b->graph));
        BATCH_CHECK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    } catch (const lbm::HipFailure &e) {
        for (int i = 0; i < n; ++i)
            if (saved[i]) b->m[i]->stream = saved[i];
        if (cs) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(cs, &g);
            if (g) (void)hipGraphDestroy(g);
        }
        release(b);
        for (hipEvent_t e2 : joins)
            if (e2) (void)hipEventDestroy(e2);
        if (fork) (void)hipEventDestroy(fork);
        if (cs) (void)hipStreamDestroy(cs);
        delete b;
        return bfail(nullptr, LB_EDEVICE, e.what);
    }
    for (hipEvent_t e : joins) (void)hipEventDestroy(e);
    (void)hipEventDestroy(fork);
    (void)hipStreamDestroy(cs);
    for (lb_handle *h : b->m) {
        h->in_batch = true;
        b->cur0.push_back(h->cur);
    }
    *out = b;
    return LB_OK;
}

int lb_batch_step(lb_batch *b, int32_t nlaunches) {
    if (!b) return LB_EINVAL;
    if (nlaunches < 0) return bfail(b, LB_EINVAL, "nlaunches must be >= 0");
    if (nlaunches == 0) return LB_OK;
    const int n = (int)b->m.size();
    for (int i = 0; i < n; ++i)  // the graph holds each member's buffers for its parity at capture
        if (b->m[i]->cur != b->cur0[i])
            return bfail(b, LB_ESTATE, "member " + std::to_string(i) + " was stepped an odd number of times outside the batch");
    try {
        // after whatever the members' own streams hold (bounced populations
        // left by steps outside the batch written out first) ...
        for (int i = 0; i < n; ++i) {
            lbm::settle_bounces(b->m[i]);
            lbm::settle_lists(b->m[i]);
            b->m[i]->flags_tracked = false;
            BATCH_CHECK(hipEventRecord(b->ev_member[i], b->m[i]->stream));
            BATCH_CHECK(hipStreamWaitEvent(b->stream, b->ev_member[i], 0));
        }
        for (int r = 0; r < nlaunches; ++r) BATCH_CHECK(hipGraphLaunch(b->exec, b->stream));
        // ... and before whatever they enqueue next
        BATCH_CHECK(hipEventRecord(b->ev_done, b->stream));
        for (int i = 0; i < n; ++i) BATCH_CHECK(hipStreamWaitEvent(b->m[i]->stream, b->ev_done, 0));
    } catch (const lbm::HipFailure &e) {
        return bfail(b, LB_EDEVICE, e.what);
    }
    for (lb_handle *h : b->m) h->step += (long long)b->k * nlaunches;
    return LB_OK;
}

int32_t lb_batch_steps_per_launch(const lb_batch *b) { return b ? b->k : 0; }

const char *lb_batch_last_error(const lb_batch *b) { return b ? b->err.c_str() : g_batch_create_error.c_str(); }

void lb_batch_destroy(lb_batch *b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    release(b);
    delete b;
}

// ---------------------------------------------------------------------------
// Autotuner: times `trial_steps` steps of every compiled kernel variant and
// fused tile on the given box and spheres, and writes the fastest into
// p->kernel and p->tile.  Each candidate is a lattice of its own, created and
// destroyed in turn (the caller must leave room for one).
// ---------------------------------------------------------------------------
int lb_autotune(lb_params *p, int32_t n, const lb_particle *parts, int32_t trial_steps, double *best_ms_per_step) {
    if (!p || trial_steps < 1 || (n > 0 && !parts)) return LB_EINVAL;
    struct Cand {
        int kernel, tx, ty, tz;
    };
    std::vector<Cand> cands;
    cands.push_back({LB_KERNEL_TWOPASS, 0, 0, 0});
    if (lbm::fused_supported(*p)) {
        // the fused sweep's tiles: 64 x TY columns (TY = 4 or 8; FP64 4) and
        // z segments of TZ planes (five extra planes start each segment)
        for (int ty : {4, 8}) {
            if (p->precision == LB_FP64 && ty != 4) continue;
            int last = 0;
            for (int tz : {32, 64, 128, 256}) {
                const int z = std::min(tz, p->nz);
                if (z == last) continue;
                last = z;
                cands.push_back({LB_KERNEL_FUSED, 64, ty, z});
            }
        }
    }
    double best = 1e300;
    Cand pick = cands[0];
    for (const Cand &c : cands) {
        lb_params q = *p;
        q.kernel = c.kernel;
        q.tile[0] = c.tx;
        q.tile[1] = c.ty;
        q.tile[2] = c.tz;
        lb_handle *h = nullptr;
        if (lb_create(&q, nullptr, nullptr, &h) != LB_OK) continue;
        int rc = n > 0 ? lb_add_particles(h, n, parts) : LB_OK;
        if (rc == LB_OK) rc = lb_step(h, 2);
        if (rc == LB_OK) rc = lb_synchronize(h);
        if (rc == LB_OK) {
            lb_enable_timing(h, 1);
            rc = lb_step(h, trial_steps);
            if (rc == LB_OK) rc = lb_synchronize(h);
            double ms = 0.0;
            int64_t cnt = 0;
            if (rc == LB_OK && lb_kernel_timing(h, 2, &ms, &cnt) == LB_OK && cnt > 0 && ms / cnt < best) {
                best = ms / cnt;
                pick = c;
            }
        }
        lb_destroy(h);
    }
    if (best == 1e300) return LB_EDEVICE;
    p->kernel = pick.kernel;
    p->tile[0] = pick.tx;
    p->tile[1] = pick.ty;
    p->tile[2] = pick.tz;
    if (best_ms_per_step) *best_ms_per_step = best;
    return LB_OK;
}

}  // extern "C"
