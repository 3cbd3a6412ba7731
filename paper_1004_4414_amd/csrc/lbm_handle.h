// Host-side state of one lattice and the launchers of its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_device.h"

struct lb_handle {
    lb_params prm{};
    lbm::DevParams dp{};
    hipStream_t stream = nullptr;
    // the pair search runs on a stream of its own, forked from `stream` at the
    // start of a step and joined before the sphere forces are summed
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_lists = nullptr;
    int device = 0;  // the device current at lb_create
    lb_allocator alloc{};
    bool have_alloc = false;
    std::string err;
    long long N = 0;
    size_t tsize = 4;  // bytes per stored population
    size_t csize = 4;  // bytes of the arithmetic type (densities, Psi, forces)

    // fluid
    void *f[2] = {nullptr, nullptr};
    int cur = 0;
    void *rho = nullptr;  // T [2][N]: densities (fluid), virtual densities (shell)
    // the densities of the previous step (swapped with rho at every step in
    // which the sweep forms bounced populations: their wall term needs them)
    void *rho_prev = nullptr;
    void *psi = nullptr;  // T [2][N]: Psi - Psi(rho_ref) of the two-pass variant
    void *fsc = nullptr;  // T [3][N]: Shan-Chen force on virtual-fluid sites
    uint32_t *info = nullptr;
    int32_t *owner = nullptr;
    int32_t *stage = nullptr;
    double *partial = nullptr;  // per-block partial sums
    int n_partial = 0;
    lbm::DevState *dstate = nullptr;
    double *fields = nullptr;  // lazily allocated output staging of lb_get_fields
    double *phi = nullptr;     // lazily allocated order parameter of the observables

    // particles
    int np = 0;
    int max_shell_cap = 0;  // the largest virtual-fluid list capacity of a sphere
    lbm::DevParticles dpart{};
    std::vector<void *> part_allocs;
    std::vector<double> h_rad, h_dens, h_color;
    std::vector<int32_t> h_prescribed;

    int kernel = LB_KERNEL_TWOPASS;
    int tile[3] = {0, 0, 0};
    int fused_tx = 64, fused_ty = 4, fused_tz = 32;  // fused-kernel tile
    int n_fused_blocks = 0;
    long long step = 0;
    bool in_batch = false;      // a batch graph holds this lattice's pointers
    // bounce-back of sphere links (see sweep_bounce in lbm_api.hip):
    // bounce_pending = the last step left bounced populations for the next
    // sweep to form; flags_tracked = the class-word flags are exactly those of
    // the last map update and chg_prev holds its change lists
    bool bounce_pending = false;
    bool flags_tracked = false;
    // lists_pending: the virtual-fluid lists of the last map update are still
    // to be built (the next step builds them on the second stream, beside its
    // density sweep; readers of the lists build them first: settle_lists)
    bool lists_pending = false;
    std::vector<void *> owned;  // every device allocation, freed by lb_destroy

    // event timing (measurement only): per kind, pairs of recorded events
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pairs[3];
    hipEvent_t timing_begin(int kind);
    void timing_end(int kind, hipEvent_t start);
};

namespace lbm {

void *dev_alloc(lb_handle *h, size_t bytes);
void one_step(lb_handle *h);  // enqueue one time step on h->stream
// write out every bounced population the last step left to the next sweep
// (before any other reader of the stored populations)
void settle_bounces(lb_handle *h);
// build the virtual-fluid lists the last step left pending (before any other
// reader of the lists or of their counts)
void settle_lists(lb_handle *h);
void launch_clear_flags(lb_handle *h);  // class-word flags of the map update, all sites
void dev_free(lb_handle *h, void *p);

// fluid (lbm_fluid.hip)
void launch_init_fluid(lb_handle *h);
void launch_density(lb_handle *h, const void *f, bool partial_sums);
void launch_finalize_mass(lb_handle *h);
void launch_shell_fill(lb_handle *h);
// calls fn(tag) with tag::type the population storage type of the precision
template <typename S>
struct StorageTag {
    using type = S;
};
template <typename Fn>
void with_storage(const lb_params &p, Fn &&fn) {
    switch (p.precision) {
    case LB_FP64: fn(StorageTag<double>{}); break;
    case LB_FP16: fn(StorageTag<__half>{}); break;
    case LB_BF16: fn(StorageTag<__hip_bfloat16>{}); break;
    default: fn(StorageTag<float>{}); break;
    }
}

// calls fn(Model<velocity_mode, eq_order>{}) for the handle's parameters
template <typename Fn>
void with_model(const lb_params &p, Fn &&fn) {
    if (p.velocity_mode == 1) {
        if (p.eq_order == 3) fn(Model<1, 3>{});
        else fn(Model<1, 2>{});
    } else {
        if (p.eq_order == 3) fn(Model<0, 3>{});
        else fn(Model<0, 2>{});
    }
}
void launch_collide_stream(lb_handle *h, const void *fin, void *fout);
void launch_wall_links(lb_handle *h, void *fout);
void launch_fields(lb_handle *h, const void *f, double *out);
void launch_sums(lb_handle *h, const void *f);
void launch_finalize_mass_n(lb_handle *h, int nblocks);

// fused single sweep (lbm_fused.hip)
bool fused_supported(const lb_params &p);
void launch_fused(lb_handle *h, const void *fin, void *fout);
void launch_fill_int(lb_handle *h, int32_t *p, long long n, int32_t v);
void launch_info_dense(lb_handle *h);
void launch_owner_reset(lb_handle *h);

// particles (lbm_particles.hip)
void launch_particle_fluid_force(lb_handle *h, void *fout);
void launch_pair_forces(lb_handle *h, hipStream_t s);
void launch_forces_total(lb_handle *h);
void launch_integrate(lb_handle *h);
void launch_map_mark(lb_handle *h);  // full classification (marks in stage[])
void launch_map_flip(lb_handle *h);  // per-step update: changed sites and events
void launch_map_fixup(lb_handle *h, void *fout);   // links next to this step's map changes, written out
void launch_materialize(lb_handle *h, void *f);    // every pending bounced population written out
void launch_cover_refill(lb_handle *h, void *fout);
void launch_map_commit(lb_handle *h, bool full);
void launch_map_info(lb_handle *h);
void launch_fold_events(lb_handle *h);  // per-sphere event counts into DevState
void launch_build_lists(lb_handle *h, bool full, hipStream_t s);

// a batch advanced by shared launches: one launch per stage of the step for
// all members (lbm_batch.hip builds it; the launchers are in lbm_fluid.hip and
// lbm_particles.hip)
constexpr int PAIR_CELLS_MIN_SPHERES = 1024;  // the cell-list pair search from this many spheres
struct BatchLaunch {
    BatchPlan plan[2];       // device tables for the two step parities (fin / fout swapped)
    int total[BM_COUNT];     // blocks of each map over all members
    int nm;
    int fin_stride;          // blocks per member of the mass total: the most fin_blocks() of any member
    int any_rows, any_flat;  // members with row-aligned addressing (nx % 64 == 0), and without
    lb_params prm;           // precision and collision model shared by the members
};
void launch_batch_fluid(const BatchLaunch &L, int parity, hipStream_t s);
void launch_batch_particles(const BatchLaunch &L, int parity, hipStream_t s);

}  // namespace lbm

#define LB_HIP_CHECK(expr)                                                            \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) throw lbm::HipFailure(#expr, hipGetErrorString(e_));    \
    } while (0)

namespace lbm {
struct HipFailure {
    std::string what;
    HipFailure(const char *expr, const char *msg) : what(std::string(expr) + ": " + msg) {}
};
}  // namespace lbm
