// C interface (include/lbm.h): parameter validation, device memory through the
// caller's allocator, stream-ordered orchestration of the kernels of one time
// step, host copies of fields and state, and deferred device-error reporting.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbm_handle.h"

using namespace lbm;

namespace lbm {

void *dev_alloc(lb_handle *h, size_t bytes) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~size_t(255);
    void *p = nullptr;
    if (h->have_alloc) {
        p = h->alloc.alloc(bytes, h->alloc.ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (!p) throw std::bad_alloc();
    h->owned.push_back(p);
    return p;
}

void dev_free(lb_handle *h, void *p) {
    if (!p) return;
    auto it = std::find(h->owned.begin(), h->owned.end(), p);
    if (it != h->owned.end()) h->owned.erase(it);
    if (h->have_alloc) h->alloc.free(p, h->alloc.ctx);
    else (void)hipFree(p);
}

}  // namespace lbm

namespace {

int fail(lb_handle *h, int code, const std::string &msg) {
    if (h) h->err = msg;
    return code;
}

#define LB_API_BEGIN try {
#define LB_API_END                                                                    \
    }                                                                                 \
    catch (const lbm::HipFailure &e) {                                                \
        return fail(h, LB_EDEVICE, e.what);                                           \
    }                                                                                 \
    catch (const std::bad_alloc &) {                                                  \
        return fail(h, LB_ENOMEM, "device allocation failed");                        \
    }

const char *kStateMagic = "LBMSTATE";
constexpr uint32_t kStateVersion = 3;

// upper bound of the lattice sites of a sphere's outermost solid layer: those
// sites lie within sqrt(2) inside the surface, so their unit cells lie in the
// shell r - sqrt(2) - sqrt(3)/2 < |x - R| < r + sqrt(3)/2
int shell_capacity(double r) {
    const double a = r + 0.8661, b = std::max(0.0, r - 1.4143 - 0.8661);
    return (int)std::ceil(4.0 / 3.0 * M_PI * (a * a * a - b * b * b)) + 32;
}

double minimg_host(double d, double L) {
    while (d > 0.5 * L) d -= L;
    while (d < -0.5 * L) d += L;
    return d;
}

unsigned nblk(long long n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

void set_dev_params(lb_handle *h) {
    const lb_params &p = h->prm;
    DevParams &d = h->dp;
    d.nx = p.nx;
    d.ny = p.ny;
    d.nz = p.nz;
    d.np = h->np;
    d.N = h->N;
    for (int c = 0; c < 2; ++c) {
        d.tau[c] = p.tau[c];
        d.rho_init[c] = p.rho_init[c];
        // FP32 keeps deviations from the rest state of the mean density, which
        // carries the small flow signal with ~50x finer resolution; FP64 keeps f
        d.rho_ref[c] = p.precision == LB_FP64 ? 0.0 : p.rho_init[c];
        d.psi_e[c] = p.rho0 * std::exp(-d.rho_ref[c] / p.rho0);
        d.inv_tau[c] = 1.0 / p.tau[c];
    }
    d.inv_rho0 = 1.0 / p.rho0;
    d.div_nx = make_fastdiv((uint32_t)p.nx);
    d.div_nxy = make_fastdiv((uint32_t)p.nx * (uint32_t)p.ny);
    d.g = p.g_br;
    d.rho0 = p.rho0;
    d.w_face = p.w_face;
    d.w_edge = p.w_edge;
    d.velocity_mode = p.velocity_mode;
    d.eq_order = p.eq_order;
    d.wall_axis = p.wall_axis;
    d.lub_mode = p.lub_mode;
    d.link_write = 1;  // set per step by the step's launcher
    d.redirect = 0;
    d.multi_bits = h->prm.link_writes == 0;  // the sweep-side bounce reads INFO_MULTI
    d.force_avg = p.force_average;
    d.any_color = 0;
    for (double c : h->h_color) d.any_color |= c != 0.0;
    for (int a = 0; a < 3; ++a) {
        d.body[a] = p.body_accel[a];
        d.wall_vel[0][a] = p.wall_vel[0][a];
        d.wall_vel[1][a] = p.wall_vel[1][a];
    }
    d.c0 = p.c0_mass_corr;
    d.k_hertz = p.k_hertz;
    d.lub_hc = p.lub_hc;
    d.lub_hmin = p.lub_hmin;
    d.nu = 0.5 * ((p.tau[0] - 0.5) + (p.tau[1] - 0.5)) / 3.0;
}

int validate_params(const lb_params *p, std::string &msg) {
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return msg = "box edges must be >= 1", LB_EINVAL;
    const long long N = (long long)p->nx * p->ny * p->nz;
    if (N > 0x7fffffffLL / 2) return msg = "box too large (sites must fit 30 bits)", LB_EINVAL;
    if (p->precision < LB_FP64 || p->precision > LB_BF16) return msg = "unknown precision", LB_EINVAL;
    for (int c = 0; c < 2; ++c)
        if (!(p->tau[c] > 0.5)) return msg = "tau must exceed 1/2", LB_EINVAL;
    if (!(p->rho0 > 0.0)) return msg = "rho0 must be positive", LB_EINVAL;
    if (p->velocity_mode != 0 && p->velocity_mode != 1) return msg = "velocity_mode must be 0 or 1", LB_EINVAL;
    if (p->eq_order != 2 && p->eq_order != 3) return msg = "eq_order must be 2 or 3", LB_EINVAL;
    if (p->lub_mode != 0 && p->lub_mode != 1) return msg = "lub_mode must be 0 or 1", LB_EINVAL;
    if (p->link_writes != 0 && p->link_writes != 1) return msg = "link_writes must be 0 or 1", LB_EINVAL;
    if (p->force_average != 0 && p->force_average != 1) return msg = "force_average must be 0 or 1", LB_EINVAL;
    if (p->wall_axis < -1 || p->wall_axis > 2) return msg = "wall_axis must be -1, 0, 1 or 2", LB_EINVAL;
    if (p->wall_axis >= 0 && (p->wall_axis == 0 ? p->nx : (p->wall_axis == 1 ? p->ny : p->nz)) < 3)
        return msg = "a box with walls needs at least 3 sites along the wall axis", LB_EINVAL;
    if (p->kernel < LB_KERNEL_AUTO || p->kernel > LB_KERNEL_TWOPASS) return msg = "unknown kernel", LB_EINVAL;
    if (!std::isfinite(p->g_br) || !std::isfinite(p->noise_amp)) return msg = "non-finite parameter", LB_EINVAL;
    return LB_OK;
}

size_t pop_bytes(int precision) {
    return precision == LB_FP64 ? 8 : (precision == LB_FP16 || precision == LB_BF16 ? 2 : 4);
}

// host conversions of stored populations
double to_double(double v) { return v; }
double to_double(float v) { return v; }
double to_double(__half v) { return (double)__half2float(v); }
double to_double(__hip_bfloat16 v) { return (double)__bfloat162float(v); }
template <typename T>
T from_double(double v);
template <>
double from_double<double>(double v) { return v; }
template <>
float from_double<float>(double v) { return (float)v; }
template <>
__half from_double<__half>(double v) { return __float2half((float)v); }
template <>
__hip_bfloat16 from_double<__hip_bfloat16>(double v) { return __float2bfloat16((float)v); }

size_t fluid_bytes(const lb_params *p) {
    const long long N = (long long)p->nx * p->ny * p->nz;
    const size_t ts = pop_bytes(p->precision), tc = p->precision == LB_FP64 ? 8 : 4;
    size_t b = 0;
    const size_t Np = padded_sites(N);
    b += 2 * (size_t)(2 * Q) * Np * ts;  // two population buffers
    b += 8 * Np * tc;                    // densities, Psi, shell force (padded to 4)
    if (p->link_writes == 0) b += 2 * Np * tc;  // densities of the previous step
    b += 3 * (size_t)N * 4;             // info, owner, stage
    b += 8 * (size_t)nblk(N) * 8 + 4096;
    return b;
}

size_t particle_bytes(const lb_params *p, int np, double max_r) {
    const size_t sc = (size_t)shell_capacity(max_r);
    const size_t cells = (size_t)((p->nx + 7) / 8) * ((p->ny + 7) / 8) * ((p->nz + 7) / 8);
    size_t b = (size_t)np * (59 * 8 + (22 + MAX_LUB_CONTACTS + CAND_CAP + NB_CAP) * 4 + MAX_LUB_CONTACTS * 32) +
               4 * cells;
    const double reach = 2.0 * max_r + std::max(p->lub_hc, NB_REACH);  // cell list of the pair search
    b += 8 * (size_t)(p->nx / reach + 1) * (size_t)(p->ny / reach + 1) * (size_t)(p->nz / reach + 1);
    b += (size_t)np * sc * (4 + 6 * 4);  // virtual-fluid sites; covered, uncovered and two steps' changed sites
    return b + 4096;
}

// rebuild the solid map, the class words and the per-sphere lists from the
// current positions without touching the fluid
void rebuild_map(lb_handle *h) {
    settle_bounces(h);  // on the map they belong to
    h->flags_tracked = false;
    launch_fold_events(h);
    launch_owner_reset(h);
    launch_fill_int(h, h->stage, h->N, STAGE_NONE);
    LB_HIP_CHECK(hipMemcpyAsync(h->dpart.Rprev, h->dpart.R, sizeof(double) * 3 * h->np, hipMemcpyDeviceToDevice,
                                h->stream));
    LB_HIP_CHECK(hipMemcpyAsync(h->dpart.Rscan, h->dpart.R, sizeof(double) * 3 * h->np, hipMemcpyDeviceToDevice,
                                h->stream));
    launch_map_mark(h);  // every sphere is classified afresh
    launch_map_commit(h, true);
    launch_info_dense(h);
    launch_fill_int(h, h->stage, h->N, STAGE_NONE);
    h->lists_pending = false;  // built afresh here
    launch_build_lists(h, true, h->stream);
}

void free_particles(lb_handle *h) {
    for (void *p : h->part_allocs) dev_free(h, p);
    h->part_allocs.clear();
    h->dpart = DevParticles{};
    h->np = 0;
}

// stored value of (component c, direction i) <-> population f: f = stored + zeta_i rho_ref^c
template <typename T>
void to_host_populations(lb_handle *h, double *out) {
    const long long N = h->N;
    std::vector<T> buf((size_t)2 * Q * padded_sites(N));  // T: the storage type
    std::vector<int32_t> own((size_t)N);
    LB_HIP_CHECK(hipMemcpyAsync(buf.data(), h->f[h->cur], buf.size() * sizeof(T), hipMemcpyDeviceToHost, h->stream));
    LB_HIP_CHECK(hipMemcpyAsync(own.data(), h->owner, own.size() * 4, hipMemcpyDeviceToHost, h->stream));
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    const int nx = h->prm.nx, ny = h->prm.ny, nz = h->prm.nz;
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < Q; ++i) {
            const double w = zeta(i) * h->dp.rho_ref[c];
            double *dst = out + (size_t)(c * Q + i) * N;
            for (int z = 0; z < nz; ++z)
                for (int y = 0; y < ny; ++y)
                    for (int x = 0; x < nx; ++x) {
                        const long long n = ((long long)z * ny + y) * nx + x;
                        const long long src = ((long long)((z - cz(i) + nz) % nz) * ny + (y - cy(i) + ny) % ny) * nx +
                                              (x - cx(i) + nx) % nx;  // f_i(x) = slot (i, x - c_i)
                        dst[n] = own[n] == OWN_FLUID ? to_double(buf[pidx(c, i, (unsigned)src)]) + w : 0.0;
                    }
        }
}

template <typename T>
void from_host_populations(lb_handle *h, const double *in) {
    const long long N = h->N;
    std::vector<T> buf((size_t)2 * Q * padded_sites(N));
    std::vector<int32_t> own((size_t)N);
    LB_HIP_CHECK(hipMemcpyAsync(own.data(), h->owner, own.size() * 4, hipMemcpyDeviceToHost, h->stream));
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    const int nx = h->prm.nx, ny = h->prm.ny, nz = h->prm.nz;
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < Q; ++i) {
            const double w = zeta(i) * h->dp.rho_ref[c];
            const double *src = in + (size_t)(c * Q + i) * N;
            for (int z = 0; z < nz; ++z)
                for (int y = 0; y < ny; ++y)
                    for (int x = 0; x < nx; ++x) {
                        const long long n = ((long long)z * ny + y) * nx + x;
                        if (own[n] != OWN_FLUID) continue;
                        const long long dst = ((long long)((z - cz(i) + nz) % nz) * ny + (y - cy(i) + ny) % ny) * nx +
                                              (x - cx(i) + nx) % nx;
                        buf[pidx(c, i, (unsigned)dst)] = from_double<T>(src[n] - w);
                    }
        }
    LB_HIP_CHECK(hipMemcpyAsync(h->f[h->cur], buf.data(), buf.size() * sizeof(T), hipMemcpyHostToDevice, h->stream));
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
}

int check_device_state(lb_handle *h) {
    DevState st;
    LB_HIP_CHECK(hipMemcpyAsync(&st, h->dstate, sizeof(st), hipMemcpyDeviceToHost, h->stream));
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    if (st.unstable) return fail(h, LB_EUNSTABLE, "the fluid mass became non-finite");
    if (st.overflow & 8) return fail(h, LB_EUNSTABLE, "a sphere moved one lattice site or more in one step");
    if (st.overflow & 7) return fail(h, LB_ECAPACITY, "a per-sphere list overflowed");
    if (st.overflow & 16) return fail(h, LB_ECAPACITY, "a sphere has more lubrication contacts than the list holds");
    return LB_OK;
}

// fused-kernel tile: 64 sites wide (a wavefront per row), ty rows (4 or 8;
// FP64 4) and a z segment of tz planes (default 64)
void choose_fused_tile(lb_handle *h) {
    const lb_params &p = h->prm;
    int ty = p.tile[1], tz = p.tile[2];
    if (ty != 4 && ty != 8) ty = 4;
    if (p.precision == LB_FP64) ty = 4;
    if (tz <= 0) tz = 64;
    h->fused_tx = 64;
    h->fused_ty = ty;
    h->fused_tz = std::max(1, std::min(tz, p.nz));
}

// Bounced populations of sphere links, Eq. (16).  The link kernel reads f*_i(x)
// from the fluid site's slot (i, x) for the momentum sums; writing the bounced
// pair into the solid site's slot (opp(i), x + c_i) is a scattered 8-byte store
// into a line the sweep wrote in full long before, per link.  With the
// two-pass sweep (sweep_bounce), the next step's density and collide sweeps
// form the pair themselves from slot (i, x), the density deviations of x of
// the bounce's step (rho_prev) and the sphere state the link kernel used,
// and the solid slot is left at the zero the sweep stored there.  The map
// update changes links: for the fluid sites within one site of a site whose
// owner changes, the fix-up writes the bounced pairs out before covering and
// refilling read or overwrite those slots, and the class-word kernel flags
// their words, so the next sweep pulls them plainly.  Readers of the stored
// populations outside the sweeps (observables, fields, checkpoints, batches,
// a full map rebuild) first write out every pending pair (settle_bounces).
// This is the lb_params.link_writes = 0 option: measured at 256^3 with 4806
// spheres, the density sweep's extra dependent loads at boundary sites (most
// wavefronts have some) cost more than the scattered stores it saves, so the
// link kernel writes the pairs by default.
bool sweep_bounce(const lb_handle *h, bool capturing) {
    return h->np > 0 && h->kernel == LB_KERNEL_TWOPASS && !capturing && h->prm.link_writes == 0;
}

void enqueue_step(lb_handle *h) {
    void *fin = h->f[h->cur], *fout = h->f[1 - h->cur];
    hipEvent_t t_step = h->timing_begin(2);
    // The pair search and forces read only the spheres' positions and
    // velocities, which nothing changes before the integration: outside a
    // stream capture they run on a second stream beside the fluid sweep and
    // the link sums (a captured step keeps them on the one stream).
    hipStreamCaptureStatus capturing = hipStreamCaptureStatusNone;
    LB_HIP_CHECK(hipStreamIsCapturing(h->stream, &capturing));
    const bool fork = h->np && capturing == hipStreamCaptureStatusNone;
    const bool sb = sweep_bounce(h, capturing != hipStreamCaptureStatusNone);
    if (!sb) settle_bounces(h);
    if (sb) {
        std::swap(h->rho, h->rho_prev);
        std::swap(h->dpart.chg, h->dpart.chg_prev);
        std::swap(h->dpart.chg_cnt, h->dpart.chg_prev_cnt);
        // without the previous update's lists every flag is cleared here (no
        // bounce is pending then: the previous step wrote its links)
        if (!h->flags_tracked) launch_clear_flags(h);
        h->dpart.track_flags = h->flags_tracked ? 1 : 0;
        h->dp.redirect = h->bounce_pending ? 1 : 0;
        h->dp.link_write = 0;
    } else {
        h->dpart.track_flags = 0;
        h->dp.redirect = 0;
        h->dp.link_write = 1;
    }
    // The virtual-fluid lists of the last map update are read first by this
    // step's virtual-fluid fill, and the density sweep does not touch what
    // they are built from: with the second stream (and the two-pass sweep)
    // they are built there, beside the density sweep (a captured step builds
    // them at its end, on the one stream).
    bool lists_beside = false;
    if (fork) {
        LB_HIP_CHECK(hipEventRecord(h->ev_fork, h->stream));
        LB_HIP_CHECK(hipStreamWaitEvent(h->side, h->ev_fork, 0));
        if (h->lists_pending) {
            launch_build_lists(h, false, h->side);
            LB_HIP_CHECK(hipEventRecord(h->ev_lists, h->side));
            h->lists_pending = false;
            lists_beside = true;
        }
        launch_pair_forces(h, h->side);
        LB_HIP_CHECK(hipEventRecord(h->ev_join, h->side));
    } else {
        settle_lists(h);
    }
    if (h->kernel == LB_KERNEL_FUSED) {
        hipEvent_t t_col = h->timing_begin(0);
        launch_fused(h, fin, fout);  // its virtual fluid comes from the class words
        h->timing_end(0, t_col);
        launch_finalize_mass_n(h, h->n_fused_blocks);
    } else {
        hipEvent_t t_den = h->timing_begin(1);
        launch_density(h, fin, true);
        h->timing_end(1, t_den);
        launch_finalize_mass(h);
        if (lists_beside) LB_HIP_CHECK(hipStreamWaitEvent(h->stream, h->ev_lists, 0));
        launch_shell_fill(h);
        hipEvent_t t_col = h->timing_begin(0);
        launch_collide_stream(h, fin, fout);
        h->timing_end(0, t_col);
    }
    launch_wall_links(h, fout);
    if (h->np) {
        launch_particle_fluid_force(h, fout);
        if (fork) LB_HIP_CHECK(hipStreamWaitEvent(h->stream, h->ev_join, 0));
        else launch_pair_forces(h, h->stream);
        launch_forces_total(h);
        launch_integrate(h);
        launch_map_flip(h);  // also clears the dirty cells (and the previous update's flags)
        if (sb) launch_map_fixup(h, fout);
        launch_cover_refill(h, fout);
        launch_map_commit(h, false);
        launch_map_info(h);
        // built beside the next step's density sweep; the fused sweep, held
        // to two wavefronts per SIMD by its registers, took 0.23 ms longer
        // with the walk beside it, so its lists are built here
        if (fork && h->kernel == LB_KERNEL_TWOPASS) h->lists_pending = true;
        else launch_build_lists(h, false, h->stream);
    }
    h->timing_end(2, t_step);
    h->cur = 1 - h->cur;
    ++h->step;
    h->bounce_pending = sb;
    h->flags_tracked = sb;
    h->dp.redirect = 0;  // other launches between steps pull plainly
    h->dp.link_write = 1;
}

void release_events(lb_handle *h) {
    for (int k = 0; k < 3; ++k) {
        for (auto &pr : h->ev_pairs[k]) {
            h->ev_pool.push_back(pr.first);
            h->ev_pool.push_back(pr.second);
        }
        h->ev_pairs[k].clear();
    }
}

}  // namespace

void lbm::one_step(lb_handle *h) { enqueue_step(h); }

void lbm::settle_bounces(lb_handle *h) {
    if (!h->bounce_pending) return;
    launch_materialize(h, h->f[h->cur]);
    h->bounce_pending = false;
}

void lbm::settle_lists(lb_handle *h) {
    if (!h->lists_pending) return;
    launch_build_lists(h, false, h->stream);
    h->lists_pending = false;
}

hipEvent_t lb_handle::timing_begin(int) {
    if (!timing) return nullptr;
    hipEvent_t e;
    if (!ev_pool.empty()) {
        e = ev_pool.back();
        ev_pool.pop_back();
    } else {
        LB_HIP_CHECK(hipEventCreate(&e));
    }
    LB_HIP_CHECK(hipEventRecord(e, stream));
    return e;
}

void lb_handle::timing_end(int kind, hipEvent_t start) {
    if (!timing || !start) return;
    hipEvent_t e;
    if (!ev_pool.empty()) {
        e = ev_pool.back();
        ev_pool.pop_back();
    } else {
        LB_HIP_CHECK(hipEventCreate(&e));
    }
    LB_HIP_CHECK(hipEventRecord(e, stream));
    ev_pairs[kind].emplace_back(start, e);
}

extern "C" {

void lb_default_params(lb_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->nx = p->ny = p->nz = 16;
    p->precision = LB_FP32;
    p->tau[0] = p->tau[1] = 1.0;
    p->g_br = 0.08;
    p->rho0 = 1.0;
    p->w_face = 4.0;
    p->w_edge = 2.0;
    p->velocity_mode = 1;
    p->eq_order = 3;
    p->rho_init[0] = p->rho_init[1] = 0.35;
    p->noise_amp = 0.01;
    p->seed = 1;
    p->wall_axis = -1;
    p->c0_mass_corr = 0.0;
    p->k_hertz = 100.0;
    p->lub_hc = 2.0 / 3.0;
    p->lub_hmin = 0.1;
    p->kernel = LB_KERNEL_AUTO;
    p->lub_mode = 1;
    p->link_writes = 1;
    p->force_average = 0;
}

// message of the last failed lb_create on this thread (lb_last_error(NULL))
thread_local std::string g_create_error = "null handle";

int lb_create(const lb_params *p, const lb_allocator *alloc, void *stream, lb_handle **out) {
    if (!p || !out) return LB_EINVAL;
    *out = nullptr;
    std::string msg;
    int rc = validate_params(p, msg);
    if (rc != LB_OK) {
        g_create_error = msg;
        return rc;
    }
    lb_handle *h = new (std::nothrow) lb_handle();
    if (!h) return LB_ENOMEM;
    h->prm = *p;
    h->stream = (hipStream_t)stream;
    if (hipGetDevice(&h->device) != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        g_create_error = "hipGetDevice failed";
        return LB_EDEVICE;
    }
    if (alloc && alloc->alloc && alloc->free) {
        h->alloc = *alloc;
        h->have_alloc = true;
    }
    h->N = (long long)p->nx * p->ny * p->nz;
    h->tsize = pop_bytes(p->precision);
    h->csize = p->precision == LB_FP64 ? 8 : 4;
    if (p->kernel == LB_KERNEL_FUSED && !fused_supported(*p)) {
        delete h;
        return LB_EINVAL;
    }
    // automatic choice: the two-pass sweep, the faster one on the boxes tried
    // (32^3 to 256^3) in FP64, FP16 and BF16 and from rest; at a developed
    // 256^3 FP32 state the fused sweep is about 1% faster (lb_autotune picks
    // per box)
    h->kernel = p->kernel == LB_KERNEL_AUTO ? LB_KERNEL_TWOPASS : p->kernel;
    for (int a = 0; a < 3; ++a) h->tile[a] = p->tile[a];
    choose_fused_tile(h);
    set_dev_params(h);
    try {
        const size_t Np = padded_sites(h->N);
        const size_t fsz = (size_t)2 * Q * Np * h->tsize;
        h->f[0] = dev_alloc(h, fsz);
        h->f[1] = dev_alloc(h, fsz);
        h->rho = dev_alloc(h, (size_t)2 * Np * h->csize);
        h->psi = dev_alloc(h, (size_t)2 * Np * h->csize);
        h->fsc = dev_alloc(h, (size_t)4 * Np * h->csize);
        h->info = (uint32_t *)dev_alloc(h, (size_t)h->N * 4);
        h->owner = (int32_t *)dev_alloc(h, (size_t)h->N * 4);
        h->stage = (int32_t *)dev_alloc(h, (size_t)h->N * 4);
        h->n_partial = (int)nblk(h->N);
        const long long nfused = (long long)((p->nx + h->fused_tx - 1) / h->fused_tx) *
                                 ((p->ny + h->fused_ty - 1) / h->fused_ty) * ((p->nz + h->fused_tz - 1) / h->fused_tz);
        h->partial = (double *)dev_alloc(h, (size_t)std::max(8LL * h->n_partial, 2 * nfused + 16) * 8);
        h->dstate = (DevState *)dev_alloc(h, sizeof(DevState));
        // the bounce's densities for the sweep-side bounce
        if (p->link_writes == 0) h->rho_prev = dev_alloc(h, (size_t)2 * Np * h->csize);
        LB_HIP_CHECK(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
        LB_HIP_CHECK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
        LB_HIP_CHECK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
        LB_HIP_CHECK(hipEventCreateWithFlags(&h->ev_lists, hipEventDisableTiming));
        LB_HIP_CHECK(hipMemsetAsync(h->dstate, 0, sizeof(DevState), h->stream));
        LB_HIP_CHECK(hipMemsetAsync(h->f[1], 0, fsz, h->stream));
        launch_fill_int(h, h->stage, h->N, STAGE_NONE);
        launch_init_fluid(h);
        LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    } catch (const lbm::HipFailure &e) {
        g_create_error = e.what;
        lb_destroy(h);
        return LB_EDEVICE;
    } catch (const std::bad_alloc &) {
        g_create_error = "device allocation failed";
        lb_destroy(h);
        return LB_ENOMEM;
    }
    *out = h;
    return LB_OK;
}

void lb_destroy(lb_handle *h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    if (h->side) {
        (void)hipStreamSynchronize(h->side);
        (void)hipStreamDestroy(h->side);
    }
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    if (h->ev_lists) (void)hipEventDestroy(h->ev_lists);
    release_events(h);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    h->ev_pool.clear();
    std::vector<void *> all = h->owned;
    for (void *p : all) dev_free(h, p);
    delete h;
}

const char *lb_last_error(const lb_handle *h) { return h ? h->err.c_str() : g_create_error.c_str(); }

int lb_add_particles(lb_handle *h, int32_t n, const lb_particle *parts) {
    if (!h) return LB_EINVAL;
    if (h->step > 0) return fail(h, LB_ESTATE, "spheres can only be added before the first step");
    if (h->in_batch) return fail(h, LB_ESTATE, "the lattice belongs to a batch");
    if (n < 0 || (n > 0 && !parts)) return fail(h, LB_EINVAL, "bad particle array");
    if (n == 0) return LB_OK;
    if (h->prm.wall_axis >= 0) return fail(h, LB_EINVAL, "spheres and walls cannot be combined");
    const int L[3] = {h->prm.nx, h->prm.ny, h->prm.nz};
    const int minL = std::min(L[0], std::min(L[1], L[2]));
    for (int k = 0; k < n; ++k) {
        const lb_particle &q = parts[k];
        if (!(q.radius > 0.0) || q.radius > 0.25 * minL || !(q.density > 0.0) || !std::isfinite(q.color))
            return fail(h, LB_EINVAL, "sphere radius must be in (0, L/4] and density positive");
        for (int a = 0; a < 3; ++a) {
            if (!(q.pos[a] >= 0.0 && q.pos[a] < L[a])) return fail(h, LB_EINVAL, "sphere centre outside the box");
            if (2 * (int)std::ceil(q.radius) + 7 > L[a]) return fail(h, LB_EINVAL, "box too small for the sphere");
        }
    }
    // all spheres: existing then new
    std::vector<double> pos, vel, om;
    LB_API_BEGIN
    const int old = h->np;
    if (old) {
        pos.resize(3 * old);
        vel.resize(3 * old);
        om.resize(3 * old);
        LB_HIP_CHECK(hipMemcpyAsync(pos.data(), h->dpart.R, 24 * old, hipMemcpyDeviceToHost, h->stream));
        LB_HIP_CHECK(hipMemcpyAsync(vel.data(), h->dpart.U, 24 * old, hipMemcpyDeviceToHost, h->stream));
        LB_HIP_CHECK(hipMemcpyAsync(om.data(), h->dpart.W, 24 * old, hipMemcpyDeviceToHost, h->stream));
        LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    }
    std::vector<double> rad = h->h_rad, dens = h->h_dens, col = h->h_color;
    std::vector<int32_t> pre = h->h_prescribed;
    for (int k = 0; k < n; ++k) {
        for (int a = 0; a < 3; ++a) {
            pos.push_back(parts[k].pos[a]);
            vel.push_back(parts[k].vel[a]);
            om.push_back(parts[k].omega[a]);
        }
        rad.push_back(parts[k].radius);
        dens.push_back(parts[k].density);
        col.push_back(parts[k].color);
        pre.push_back(parts[k].prescribed ? 1 : 0);
    }
    const int tot = old + n;
    // overlap test, minimum image, against spheres on a coarse cell grid
    {
        double rmax = *std::max_element(rad.begin(), rad.end());
        int nc[3];
        for (int a = 0; a < 3; ++a) nc[a] = std::max(1, (int)(L[a] / (2 * rmax)));
        // fewer than 3 cells along an axis: one cell holds everything (brute force)
        if (nc[0] < 3 || nc[1] < 3 || nc[2] < 3) nc[0] = nc[1] = nc[2] = 1;
        std::vector<std::vector<int>> cells((size_t)nc[0] * nc[1] * nc[2]);
        auto cell_of = [&](int p, int a) { return std::min(nc[a] - 1, (int)(pos[3 * p + a] / L[a] * nc[a])); };
        for (int p = 0; p < tot; ++p)
            cells[((size_t)cell_of(p, 2) * nc[1] + cell_of(p, 1)) * nc[0] + cell_of(p, 0)].push_back(p);
        for (int p = old; p < tot; ++p) {
            const int c0 = cell_of(p, 0), c1 = cell_of(p, 1), c2 = cell_of(p, 2);
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (nc[0] == 1 && (dx || dy || dz)) continue;
                        const size_t ci = ((size_t)((c2 + dz + nc[2]) % nc[2]) * nc[1] + (c1 + dy + nc[1]) % nc[1]) *
                                              nc[0] + (c0 + dx + nc[0]) % nc[0];
                        for (int q : cells[ci]) {
                            if (q == p || (q >= old && q > p)) continue;
                            double d2 = 0.0;
                            for (int a = 0; a < 3; ++a) {
                                const double d = minimg_host(pos[3 * q + a] - pos[3 * p + a], L[a]);
                                d2 += d * d;
                            }
                            const double rs = rad[p] + rad[q];
                            if (d2 <= rs * rs) return fail(h, LB_EOVERLAP, "spheres overlap");
                        }
                    }
        }
    }
    // per-sphere list capacities
    std::vector<int32_t> shell_off(tot), shell_cap(tot), ev_off(tot), ev_cap(tot);
    long long ssum = 0, esum = 0;
    for (int p = 0; p < tot; ++p) {
        const int sc = shell_capacity(rad[p]);
        shell_off[p] = (int32_t)ssum;
        shell_cap[p] = sc;
        ssum += sc;
        ev_off[p] = (int32_t)esum;
        ev_cap[p] = sc;
        esum += sc;
    }
    if (ssum > 0x7fffffffLL) return fail(h, LB_EINVAL, "too many spheres for the list capacity");
    launch_fold_events(h);  // the old spheres' event counts into the totals first
    free_particles(h);
    h->np = tot;
    h->max_shell_cap = 0;
    for (int p = 0; p < tot; ++p) h->max_shell_cap = std::max(h->max_shell_cap, (int)shell_cap[p]);
    DevParticles &D = h->dpart;
    double *dbl = (double *)dev_alloc(h, sizeof(double) * 34 * tot);
    int32_t *i32 = (int32_t *)dev_alloc(h, sizeof(int32_t) * 10 * tot);
    h->part_allocs.push_back(dbl);
    h->part_allocs.push_back(i32);
    D.R = dbl;
    D.U = dbl + 3 * tot;
    D.W = dbl + 6 * tot;
    D.Rprev = dbl + 9 * tot;
    D.Ffl = dbl + 12 * tot;
    D.Tfl = dbl + 15 * tot;
    D.Ftot = dbl + 18 * tot;
    D.Ttot = dbl + 21 * tot;
    D.P = dbl + 24 * tot;
    D.PT = dbl + 27 * tot;
    D.rad = dbl + 30 * tot;
    D.mass = dbl + 31 * tot;
    D.inertia = dbl + 32 * tot;
    D.color = dbl + 33 * tot;
    D.prescribed = i32;
    D.link_cnt = i32 + tot;
    D.shell_off = i32 + 2 * tot;
    D.shell_cap = i32 + 3 * tot;
    D.shell_cnt = i32 + 4 * tot;
    D.ev_off = i32 + 5 * tot;
    D.ev_cap = i32 + 6 * tot;
    D.cov_cnt = i32 + 7 * tot;
    D.unc_cnt = i32 + 8 * tot;
    D.chg_cnt = i32 + 9 * tot;
    D.cgx = (h->prm.nx + (1 << CELL_SHIFT) - 1) >> CELL_SHIFT;
    D.cgy = (h->prm.ny + (1 << CELL_SHIFT) - 1) >> CELL_SHIFT;
    D.cgz = (h->prm.nz + (1 << CELL_SHIFT) - 1) >> CELL_SHIFT;
    D.dirty = (int32_t *)dev_alloc(h, sizeof(int32_t) * (size_t)D.cgx * D.cgy * D.cgz);
    D.lbox = (int32_t *)dev_alloc(h, sizeof(int32_t) * 6 * (size_t)tot);
    D.ncont = (int32_t *)dev_alloc(h, sizeof(int32_t) * (size_t)tot);
    D.cont = (int32_t *)dev_alloc(h, sizeof(int32_t) * MAX_LUB_CONTACTS * (size_t)tot);
    D.vs = (double *)dev_alloc(h, sizeof(double) * 3 * (size_t)tot);
    D.Fprev = (double *)dev_alloc(h, sizeof(double) * 6 * (size_t)tot);
    LB_HIP_CHECK(hipMemsetAsync(D.Fprev, 0xff, sizeof(double) * 6 * (size_t)tot, h->stream));  // NaN: none yet
    h->part_allocs.push_back(D.Fprev);
    D.Rscan = (double *)dev_alloc(h, sizeof(double) * 3 * (size_t)tot);
    D.margin = (double *)dev_alloc(h, sizeof(double) * (size_t)tot);
    D.nnbr = (int32_t *)dev_alloc(h, sizeof(int32_t) * (size_t)tot);
    D.nbr = (int32_t *)dev_alloc(h, sizeof(int32_t) * NB_CAP * (size_t)tot);
    D.ncand = (int32_t *)dev_alloc(h, sizeof(int32_t) * (size_t)tot);
    D.cand = (int32_t *)dev_alloc(h, sizeof(int32_t) * CAND_CAP * (size_t)tot);
    h->part_allocs.push_back(D.ncand);
    h->part_allocs.push_back(D.cand);
    h->part_allocs.push_back(D.Rscan);
    h->part_allocs.push_back(D.margin);
    h->part_allocs.push_back(D.nnbr);
    h->part_allocs.push_back(D.nbr);
    D.cont_c = (double *)dev_alloc(h, sizeof(double) * MAX_LUB_CONTACTS * (size_t)tot);
    D.cont_n = (double *)dev_alloc(h, sizeof(double) * 3 * MAX_LUB_CONTACTS * (size_t)tot);
    h->part_allocs.push_back(D.cont_c);
    h->part_allocs.push_back(D.cont_n);
    h->part_allocs.push_back(D.dirty);
    h->part_allocs.push_back(D.lbox);
    h->part_allocs.push_back(D.ncont);
    h->part_allocs.push_back(D.cont);
    h->part_allocs.push_back(D.vs);
    {  // cell list of the pair search: cells at least 2 r_max + h_c wide
        const double rmax = *std::max_element(rad.begin(), rad.end());
        // (NB_REACH: the neighbours of the map update are found as well)
        const double reach = 2.0 * rmax + std::max(h->prm.lub_hc, NB_REACH) + 1e-5;
        int pg[3];
        for (int a = 0; a < 3; ++a) pg[a] = reach > 0.0 ? (int)(L[a] / reach) : 1;
        if (pg[0] >= 3 && pg[1] >= 3 && pg[2] >= 3 && (long long)pg[0] * pg[1] * pg[2] <= (1 << 22)) {
            D.pgx = pg[0];
            D.pgy = pg[1];
            D.pgz = pg[2];
            const size_t nc = (size_t)pg[0] * pg[1] * pg[2];
            D.pc_cnt = (int32_t *)dev_alloc(h, sizeof(int32_t) * nc);
            D.pc_start = (int32_t *)dev_alloc(h, sizeof(int32_t) * (nc + 1));
            D.pc_items = (int32_t *)dev_alloc(h, sizeof(int32_t) * (size_t)tot);
            D.pc_of = (int32_t *)dev_alloc(h, sizeof(int32_t) * (size_t)tot);
            LB_HIP_CHECK(hipMemsetAsync(D.pc_cnt, 0, sizeof(int32_t) * nc, h->stream));
            h->part_allocs.push_back(D.pc_cnt);
            h->part_allocs.push_back(D.pc_start);
            h->part_allocs.push_back(D.pc_items);
            h->part_allocs.push_back(D.pc_of);
        } else {
            D.pgx = D.pgy = D.pgz = 0;
            D.pc_cnt = D.pc_start = D.pc_items = D.pc_of = nullptr;
        }
    }
    D.shell = (int32_t *)dev_alloc(h, sizeof(int32_t) * ssum);
    D.cov = (int32_t *)dev_alloc(h, sizeof(int32_t) * esum);
    D.unc = (int32_t *)dev_alloc(h, sizeof(int32_t) * esum);
    D.chg = (int32_t *)dev_alloc(h, sizeof(int32_t) * 2 * esum);
    D.chg_prev = (int32_t *)dev_alloc(h, sizeof(int32_t) * 2 * esum);
    D.chg_prev_cnt = (int32_t *)dev_alloc(h, sizeof(int32_t) * (size_t)tot);
    D.Rl = (double *)dev_alloc(h, sizeof(double) * 9 * (size_t)tot);
    D.Ul = D.Rl + 3 * tot;
    D.Wl = D.Rl + 6 * tot;
    D.track_flags = 0;
    LB_HIP_CHECK(hipMemsetAsync(D.chg_prev_cnt, 0, sizeof(int32_t) * (size_t)tot, h->stream));
    h->part_allocs.push_back(D.chg_prev);
    h->part_allocs.push_back(D.chg_prev_cnt);
    h->part_allocs.push_back(D.Rl);
    D.evtot = (unsigned long long *)dev_alloc(h, sizeof(unsigned long long) * 3 * (size_t)tot);
    LB_HIP_CHECK(hipMemsetAsync(D.evtot, 0, sizeof(unsigned long long) * 3 * (size_t)tot, h->stream));
    h->part_allocs.push_back(D.evtot);
    h->part_allocs.push_back(D.shell);
    h->part_allocs.push_back(D.cov);
    h->part_allocs.push_back(D.unc);
    h->part_allocs.push_back(D.chg);
    // host image of the double block
    std::vector<double> hd((size_t)34 * tot, 0.0);
    for (int p = 0; p < tot; ++p) {
        for (int a = 0; a < 3; ++a) {
            hd[3 * p + a] = pos[3 * p + a];
            hd[3 * tot + 3 * p + a] = vel[3 * p + a];
            hd[6 * tot + 3 * p + a] = om[3 * p + a];
            hd[9 * tot + 3 * p + a] = pos[3 * p + a];
        }
        const double m = dens[p] * (4.0 / 3.0) * M_PI * rad[p] * rad[p] * rad[p];
        hd[30 * tot + p] = rad[p];
        hd[31 * tot + p] = m;
        hd[32 * tot + p] = 0.4 * m * rad[p] * rad[p];
        hd[33 * tot + p] = col[p];
    }
    std::vector<int32_t> hi((size_t)10 * tot, 0);
    for (int p = 0; p < tot; ++p) {
        hi[p] = pre[p];
        hi[2 * tot + p] = shell_off[p];
        hi[3 * tot + p] = shell_cap[p];
        hi[5 * tot + p] = ev_off[p];
        hi[6 * tot + p] = ev_cap[p];
    }
    LB_HIP_CHECK(hipMemcpyAsync(dbl, hd.data(), hd.size() * 8, hipMemcpyHostToDevice, h->stream));
    LB_HIP_CHECK(hipMemcpyAsync(i32, hi.data(), hi.size() * 4, hipMemcpyHostToDevice, h->stream));
    h->h_rad = rad;
    h->h_dens = dens;
    h->h_color = col;
    h->h_prescribed = pre;
    set_dev_params(h);
    rebuild_map(h);  // the fluid inside the spheres is no longer read: it is removed
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    return check_device_state(h);
    LB_API_END
}

int lb_step(lb_handle *h, int32_t nsteps) {
    if (!h) return LB_EINVAL;
    if (nsteps < 0) return fail(h, LB_EINVAL, "nsteps must be >= 0");
    LB_API_BEGIN
    for (int s = 0; s < nsteps; ++s) enqueue_step(h);
    return LB_OK;
    LB_API_END
}

int lb_synchronize(lb_handle *h) {
    if (!h) return LB_EINVAL;
    LB_API_BEGIN
    settle_lists(h);  // their overflow check belongs to the steps taken
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    return check_device_state(h);
    LB_API_END
}

int lb_observables(lb_handle *h, lb_observables_t *out) {
    if (!h || !out) return LB_EINVAL;
    LB_API_BEGIN
    settle_bounces(h);
    settle_lists(h);
    std::memset(out, 0, sizeof(*out));
    launch_sums(h, h->f[h->cur]);
    launch_fold_events(h);
    std::vector<double> part((size_t)5 * h->n_partial);
    LB_HIP_CHECK(hipMemcpyAsync(part.data(), h->partial, part.size() * 8, hipMemcpyDeviceToHost, h->stream));
    DevState st;
    LB_HIP_CHECK(hipMemcpyAsync(&st, h->dstate, sizeof(st), hipMemcpyDeviceToHost, h->stream));
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    for (int b = 0; b < h->n_partial; ++b) {
        out->mass[0] += part[5 * b];
        out->mass[1] += part[5 * b + 1];
        for (int a = 0; a < 3; ++a) out->fluid_momentum[a] += part[5 * b + 2 + a];
    }
    out->step = h->step;
    out->n_particles = h->np;
    out->unstable = st.unstable;
    out->covered_total = (int64_t)st.covered_total;
    out->uncovered_total = (int64_t)st.uncovered_total;
    out->refill_fallback = (int64_t)st.refill_fallback;
    if (h->np) {
        const int np = h->np;
        std::vector<double> U(3 * np), P(3 * np);
        std::vector<int32_t> lc(np), sc(np);
        LB_HIP_CHECK(hipMemcpyAsync(U.data(), h->dpart.U, 24 * np, hipMemcpyDeviceToHost, h->stream));
        LB_HIP_CHECK(hipMemcpyAsync(P.data(), h->dpart.P, 24 * np, hipMemcpyDeviceToHost, h->stream));
        LB_HIP_CHECK(hipMemcpyAsync(lc.data(), h->dpart.link_cnt, 4 * np, hipMemcpyDeviceToHost, h->stream));
        LB_HIP_CHECK(hipMemcpyAsync(sc.data(), h->dpart.shell_cnt, 4 * np, hipMemcpyDeviceToHost, h->stream));
        LB_HIP_CHECK(hipStreamSynchronize(h->stream));
        for (int p = 0; p < np; ++p) {
            const double m = h->h_dens[p] * (4.0 / 3.0) * M_PI * h->h_rad[p] * h->h_rad[p] * h->h_rad[p];
            for (int a = 0; a < 3; ++a) {
                out->particle_momentum[a] += m * U[3 * p + a];
                out->pending_impulse[a] += P[3 * p + a];
            }
            out->n_links += lc[p];
            out->n_shell += sc[p];
        }
    }
    return check_device_state(h);
    LB_API_END
}

int lb_get_fields(lb_handle *h, double *rho, double *j, double *force, double *u) {
    if (!h) return LB_EINVAL;
    LB_API_BEGIN
    settle_bounces(h);
    settle_lists(h);  // the virtual-fluid fill below reads them
    const long long N = h->N;
    if (!h->fields) h->fields = (double *)dev_alloc(h, sizeof(double) * 17 * N);
    launch_density(h, h->f[h->cur], false);
    launch_shell_fill(h);
    launch_fields(h, h->f[h->cur], h->fields);
    if (rho) LB_HIP_CHECK(hipMemcpyAsync(rho, h->fields, 16 * N, hipMemcpyDeviceToHost, h->stream));
    if (j) LB_HIP_CHECK(hipMemcpyAsync(j, h->fields + 2 * N, 48 * N, hipMemcpyDeviceToHost, h->stream));
    if (force) LB_HIP_CHECK(hipMemcpyAsync(force, h->fields + 8 * N, 48 * N, hipMemcpyDeviceToHost, h->stream));
    if (u) LB_HIP_CHECK(hipMemcpyAsync(u, h->fields + 14 * N, 24 * N, hipMemcpyDeviceToHost, h->stream));
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    return check_device_state(h);
    LB_API_END
}

int lb_get_populations(lb_handle *h, double *f) {
    if (!h || !f) return LB_EINVAL;
    LB_API_BEGIN
    settle_bounces(h);
    with_storage(h->prm, [&](auto tag) { to_host_populations<typename decltype(tag)::type>(h, f); });
    return LB_OK;
    LB_API_END
}

int lb_set_populations(lb_handle *h, const double *f) {
    if (!h || !f) return LB_EINVAL;
    LB_API_BEGIN
    h->bounce_pending = false;  // the given populations replace every slot a sweep reads
    with_storage(h->prm, [&](auto tag) { from_host_populations<typename decltype(tag)::type>(h, f); });
    return LB_OK;
    LB_API_END
}

int lb_get_owner(lb_handle *h, int32_t *owner) {
    if (!h || !owner) return LB_EINVAL;
    LB_API_BEGIN
    LB_HIP_CHECK(hipMemcpyAsync(owner, h->owner, 4 * h->N, hipMemcpyDeviceToHost, h->stream));
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    return LB_OK;
    LB_API_END
}

int lb_num_particles(const lb_handle *h, int32_t *n) {
    if (!h || !n) return LB_EINVAL;
    *n = h->np;
    return LB_OK;
}

int lb_get_particles(lb_handle *h, lb_particle_state *out) {
    if (!h || (!out && h->np)) return LB_EINVAL;
    if (!h->np) return LB_OK;
    LB_API_BEGIN
    const int np = h->np;
    std::vector<double> d((size_t)34 * np);
    LB_HIP_CHECK(hipMemcpyAsync(d.data(), h->dpart.R, d.size() * 8, hipMemcpyDeviceToHost, h->stream));
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    for (int p = 0; p < np; ++p)
        for (int a = 0; a < 3; ++a) {
            out[p].pos[a] = d[3 * p + a];
            out[p].vel[a] = d[3 * np + 3 * p + a];
            out[p].omega[a] = d[6 * np + 3 * p + a];
            out[p].force_fluid[a] = d[12 * np + 3 * p + a];
            out[p].torque_fluid[a] = d[15 * np + 3 * p + a];
            out[p].force_total[a] = d[18 * np + 3 * p + a];
            out[p].torque_total[a] = d[21 * np + 3 * p + a];
            out[p].pending_impulse[a] = d[24 * np + 3 * p + a];
            out[p].pending_angular[a] = d[27 * np + 3 * p + a];
        }
    return LB_OK;
    LB_API_END
}

int lb_set_particle_state(lb_handle *h, const double *state) {
    if (!h || (!state && h->np)) return LB_EINVAL;
    if (!h->np) return LB_OK;
    LB_API_BEGIN
    const int np = h->np;
    const int L[3] = {h->prm.nx, h->prm.ny, h->prm.nz};
    std::vector<double> R(3 * np), U(3 * np), W(3 * np), P(3 * np), PT(3 * np);
    for (int p = 0; p < np; ++p)
        for (int a = 0; a < 3; ++a) {
            R[3 * p + a] = state[15 * p + a];
            U[3 * p + a] = state[15 * p + 3 + a];
            W[3 * p + a] = state[15 * p + 6 + a];
            P[3 * p + a] = state[15 * p + 9 + a];
            PT[3 * p + a] = state[15 * p + 12 + a];
            if (!(R[3 * p + a] >= 0.0 && R[3 * p + a] < L[a]))
                return fail(h, LB_EINVAL, "sphere centre outside the box");
        }
    LB_HIP_CHECK(hipMemcpyAsync(h->dpart.R, R.data(), 24 * np, hipMemcpyHostToDevice, h->stream));
    LB_HIP_CHECK(hipMemcpyAsync(h->dpart.U, U.data(), 24 * np, hipMemcpyHostToDevice, h->stream));
    LB_HIP_CHECK(hipMemcpyAsync(h->dpart.W, W.data(), 24 * np, hipMemcpyHostToDevice, h->stream));
    LB_HIP_CHECK(hipMemcpyAsync(h->dpart.P, P.data(), 24 * np, hipMemcpyHostToDevice, h->stream));
    LB_HIP_CHECK(hipMemcpyAsync(h->dpart.PT, PT.data(), 24 * np, hipMemcpyHostToDevice, h->stream));
    LB_HIP_CHECK(hipMemsetAsync(h->dpart.Fprev, 0xff, 48 * (size_t)np, h->stream));  // no previous step
    rebuild_map(h);
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    return check_device_state(h);
    LB_API_END
}

int lb_particle_counts(lb_handle *h, int32_t *links, int32_t *shell) {
    if (!h) return LB_EINVAL;
    if (!h->np) return LB_OK;
    LB_API_BEGIN
    settle_lists(h);
    if (links)
        LB_HIP_CHECK(hipMemcpyAsync(links, h->dpart.link_cnt, 4 * h->np, hipMemcpyDeviceToHost, h->stream));
    if (shell)
        LB_HIP_CHECK(hipMemcpyAsync(shell, h->dpart.shell_cnt, 4 * h->np, hipMemcpyDeviceToHost, h->stream));
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    return LB_OK;
    LB_API_END
}

// checkpoint layout: magic[8], version, np (u32 each), the lb_params the
// lattice was created with, step (i64), DevState, populations (raw storage
// type), then per sphere R U W P PT (15 doubles) radius density colour (3
// doubles) the previous step's fluid force and torque (6 doubles) prescribed
// (i32)
int lb_get_state(lb_handle *h, void *buf, size_t *bytes) {
    if (!h || !bytes) return LB_EINVAL;
    const size_t fsz = (size_t)2 * Q * padded_sites(h->N) * h->tsize;
    const size_t need = 8 + 2 * 4 + sizeof(lb_params) + 8 + sizeof(DevState) + fsz + (size_t)h->np * (24 * 8 + 4);
    if (!buf) {
        *bytes = need;
        return LB_OK;
    }
    if (*bytes < need) return fail(h, LB_EINVAL, "checkpoint buffer too small");
    LB_API_BEGIN
    char *o = (char *)buf;
    std::memcpy(o, kStateMagic, 8);
    o += 8;
    const uint32_t hdr[2] = {kStateVersion, (uint32_t)h->np};
    std::memcpy(o, hdr, sizeof(hdr));
    o += sizeof(hdr);
    std::memcpy(o, &h->prm, sizeof(lb_params));
    o += sizeof(lb_params);
    const int64_t st = h->step;
    std::memcpy(o, &st, 8);
    o += 8;
    settle_bounces(h);
    launch_fold_events(h);
    LB_HIP_CHECK(hipMemcpyAsync(o, h->dstate, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    o += sizeof(DevState);
    LB_HIP_CHECK(hipMemcpyAsync(o, h->f[h->cur], fsz, hipMemcpyDeviceToHost, h->stream));
    o += fsz;
    if (h->np) {
        const int np = h->np;
        std::vector<double> d((size_t)34 * np), fp((size_t)6 * np);
        LB_HIP_CHECK(hipMemcpyAsync(d.data(), h->dpart.R, d.size() * 8, hipMemcpyDeviceToHost, h->stream));
        LB_HIP_CHECK(hipMemcpyAsync(fp.data(), h->dpart.Fprev, fp.size() * 8, hipMemcpyDeviceToHost, h->stream));
        LB_HIP_CHECK(hipStreamSynchronize(h->stream));
        const int blocks[5] = {0, 3, 6, 24, 27};
        for (int p = 0; p < np; ++p) {
            double v[24];
            for (int b = 0; b < 5; ++b)
                for (int a = 0; a < 3; ++a) v[3 * b + a] = d[(size_t)blocks[b] * np + 3 * p + a];
            v[15] = h->h_rad[p];
            v[16] = h->h_dens[p];
            v[17] = h->h_color[p];
            for (int k = 0; k < 6; ++k) v[18 + k] = fp[(size_t)6 * p + k];
            std::memcpy(o, v, sizeof(v));
            o += sizeof(v);
            const int32_t pr = h->h_prescribed[p];
            std::memcpy(o, &pr, 4);
            o += 4;
        }
    }
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    *bytes = need;
    return LB_OK;
    LB_API_END
}

// the parameters that fix the stored state and the model it follows (the
// initial-noise draw and the kernel choice do not)
static bool same_model(const lb_params &a, const lb_params &b) {
    bool eq = a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.precision == b.precision && a.g_br == b.g_br &&
              a.rho0 == b.rho0 && a.w_face == b.w_face && a.w_edge == b.w_edge &&
              a.velocity_mode == b.velocity_mode && a.eq_order == b.eq_order && a.wall_axis == b.wall_axis &&
              a.c0_mass_corr == b.c0_mass_corr && a.k_hertz == b.k_hertz && a.lub_hc == b.lub_hc &&
              a.lub_hmin == b.lub_hmin && a.lub_mode == b.lub_mode && a.force_average == b.force_average;
    for (int c = 0; c < 2; ++c) eq = eq && a.tau[c] == b.tau[c] && a.rho_init[c] == b.rho_init[c];
    for (int k = 0; k < 3; ++k)
        eq = eq && a.body_accel[k] == b.body_accel[k] && a.wall_vel[0][k] == b.wall_vel[0][k] &&
             a.wall_vel[1][k] == b.wall_vel[1][k];
    return eq;
}

int lb_set_state(lb_handle *h, const void *buf, size_t bytes) {
    if (!h || !buf) return LB_EINVAL;
    if (h->in_batch) return fail(h, LB_ESTATE, "the lattice belongs to a batch");
    const char *in = (const char *)buf;
    const size_t head = 8 + 2 * 4 + sizeof(lb_params) + 8 + sizeof(DevState);
    if (bytes < head || std::memcmp(in, kStateMagic, 8) != 0) return fail(h, LB_EINVAL, "not a checkpoint");
    uint32_t hdr[2];
    std::memcpy(hdr, in + 8, sizeof(hdr));
    if (hdr[0] != kStateVersion) return fail(h, LB_EINVAL, "checkpoint of another format version");
    lb_params saved;
    std::memcpy(&saved, in + 16, sizeof(lb_params));
    if (!same_model(saved, h->prm))
        return fail(h, LB_EINVAL, "checkpoint of a lattice with other parameters (box, precision or model)");
    const int np = (int)hdr[1];
    const size_t fsz = (size_t)2 * Q * padded_sites(h->N) * h->tsize;
    if (bytes < head + fsz + (size_t)np * (24 * 8 + 4)) return fail(h, LB_EINVAL, "truncated checkpoint");
    const char *p = in + 16 + sizeof(lb_params);
    int64_t st;
    std::memcpy(&st, p, 8);
    p += 8;
    const char *dstate = p;
    p += sizeof(DevState);
    const char *pops = p;
    p += fsz;
    // the spheres' fixed properties as stored
    std::vector<lb_particle> parts(np);
    {
        const char *q = p;
        for (int k = 0; k < np; ++k) {
            double v[24];
            std::memcpy(v, q, sizeof(v));
            q += sizeof(v);
            int32_t pr;
            std::memcpy(&pr, q, 4);
            q += 4;
            for (int a = 0; a < 3; ++a) {
                parts[k].pos[a] = v[a];
                parts[k].vel[a] = v[3 + a];
                parts[k].omega[a] = v[6 + a];
            }
            parts[k].radius = v[15];
            parts[k].density = v[16];
            parts[k].color = v[17];
            parts[k].prescribed = pr;
        }
    }
    if (np == h->np) {
        for (int k = 0; k < np; ++k)
            if (parts[k].radius != h->h_rad[k] || parts[k].density != h->h_dens[k] ||
                parts[k].color != h->h_color[k] || (parts[k].prescribed != 0) != (h->h_prescribed[k] != 0))
                return fail(h, LB_EINVAL, "checkpoint spheres differ in radius, density, colour or motion");
    } else if (!(h->step == 0 && h->np == 0 && np > 0)) {
        return fail(h, LB_ESTATE, "checkpoint has a different number of spheres");
    }
    LB_API_BEGIN
    // spheres: a lattice without any is given the checkpoint's as a fresh addition
    if (np != h->np) {
        const int rc = lb_add_particles(h, np, parts.data());
        if (rc != LB_OK) return rc;
    }
    std::vector<double> fp((size_t)6 * np);  // read by the copy below until the final synchronisation
    if (np) {
        std::vector<double> s((size_t)15 * np);
        const char *q = p;
        for (int k = 0; k < np; ++k) {
            std::memcpy(&s[15 * k], q, 15 * 8);
            std::memcpy(&fp[6 * k], q + 18 * 8, 6 * 8);
            q += 24 * 8 + 4;
        }
        const int rc = lb_set_particle_state(h, s.data());
        if (rc != LB_OK) return rc;
        LB_HIP_CHECK(hipMemcpyAsync(h->dpart.Fprev, fp.data(), fp.size() * 8, hipMemcpyHostToDevice, h->stream));
    }
    LB_HIP_CHECK(hipMemcpyAsync(h->f[h->cur], pops, fsz, hipMemcpyHostToDevice, h->stream));
    h->bounce_pending = false;  // a checkpoint holds every bounced population in its slot
    LB_HIP_CHECK(hipMemcpyAsync(h->dstate, dstate, sizeof(DevState), hipMemcpyHostToDevice, h->stream));
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    h->step = st;
    return LB_OK;
    LB_API_END
}

int lb_enable_timing(lb_handle *h, int32_t enable) {
    if (!h) return LB_EINVAL;
    LB_API_BEGIN
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    release_events(h);
    h->timing = enable != 0;
    return LB_OK;
    LB_API_END
}

int lb_kernel_timing(lb_handle *h, int32_t which, double *ms, int64_t *launches) {
    if (!h || which < 0 || which > 2 || !ms || !launches) return LB_EINVAL;
    LB_API_BEGIN
    LB_HIP_CHECK(hipStreamSynchronize(h->stream));
    double tot = 0.0;
    for (auto &pr : h->ev_pairs[which]) {
        float t = 0.f;
        LB_HIP_CHECK(hipEventElapsedTime(&t, pr.first, pr.second));
        tot += t;
    }
    *ms = tot;
    *launches = (int64_t)h->ev_pairs[which].size();
    return LB_OK;
    LB_API_END
}

int lb_contact_angle_to_color(double theta_deg, double *color) {
    if (!color || !(theta_deg >= 0.0 && theta_deg <= 180.0)) return LB_EINVAL;
    *color = (theta_deg - 90.0) / 442.0;
    return LB_OK;
}

int lb_footprint_bytes(const lb_params *p, int32_t n_particles, double max_radius, size_t *bytes) {
    if (!p || !bytes || n_particles < 0) return LB_EINVAL;
    std::string msg;
    const int rc = validate_params(p, msg);
    if (rc != LB_OK) return rc;
    *bytes = fluid_bytes(p) + (n_particles ? particle_bytes(p, n_particles, max_radius) : 0);
    return LB_OK;
}

}  // extern "C"
