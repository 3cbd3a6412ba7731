// Fluid kernels for gfx950: initial state, densities, virtual fluid,
// Shan-Chen force, BGK collision with the velocity shift and push streaming
// with moving bounce-back (Secs. II-IV of Jansen & Harting), plus the field
// and sum kernels behind the observables.
//
// Storage: populations SoA f[c][i][n] (n = (z*ny + y)*nx + x), one plane per
// component and direction, so a wavefront's 64 lanes touch 64 consecutive
// sites of one plane.  The stored state is the post-streaming f(t); a step
// reads it at the site, collides and pushes f* to x + c_i in the other buffer
// (or bounces it back into the site when x + c_i is solid).
#include "lbm_handle.h"

namespace lbm {

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood 2014): k-th output of the generator seeded
// with s is mix(s + (k+1) * 0x9E3779B97F4A7C15).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_init_owner(DevParams P, int32_t *owner) {
    const long long n = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= P.N) return;
    int x, y, z;
    site_xyz(n, P, x, y, z);
    int32_t o = OWN_FLUID;
    if (P.wall_axis >= 0) {
        const int pos = P.wall_axis == 0 ? x : (P.wall_axis == 1 ? y : z);
        const int L = P.wall_axis == 0 ? P.nx : (P.wall_axis == 1 ? P.ny : P.nz);
        if (pos == 0) o = OWN_WALL_LO;
        else if (pos == L - 1) o = OWN_WALL_HI;
    }
    owner[n] = o;
}

// initial densities rho^c = rho_init^c + noise (2U - 1), f = zeta_i rho^c,
// stored as f - zeta_i rho_ref^c
template <typename T>
__global__ void k_init_fluid(DevParams P, uint64_t seed, double noise, const int32_t *__restrict__ owner,
                             T *__restrict__ f) {
#pragma clang fp contract(off)
    const long long n = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= P.N) return;
    const bool fluid = owner[n] == OWN_FLUID;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const double U = (double)(splitmix64_at(seed, 2ull * (unsigned long long)n + c) >> 11) *
                         (1.0 / 9007199254740992.0);
        const double r = P.rho_init[c] + noise * (2.0 * U - 1.0);
#pragma unroll
        for (int i = 0; i < Q; ++i)
            f[(long long)(c * Q + i) * P.N + n] = fluid ? (T)(zeta(i) * r - zeta(i) * P.rho_ref[c]) : (T)0;
    }
}

__global__ void k_info_dense(DevParams P, const int32_t *__restrict__ owner, uint32_t *__restrict__ info) {
    const long long n = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= P.N) return;
    info[n] = compute_info(n, P, owner);
}

__global__ void k_owner_reset(DevParams P, int32_t *owner) {
    const long long n = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= P.N) return;
    if (owner[n] >= 0) owner[n] = OWN_FLUID;
}

__global__ void k_fill_int(int32_t *p, long long n, int32_t v) {
    const long long k = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (k < n) p[k] = v;
}

template <typename T>
__global__ void k_zero_solid(DevParams P, const int32_t *__restrict__ owner, T *__restrict__ f) {
    const long long n = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= P.N || owner[n] == OWN_FLUID) return;
    for (int k = 0; k < 2 * Q; ++k) f[(long long)k * P.N + n] = (T)0;
}

// ---------------------------------------------------------------------------
// density deviations rho^c - rho_ref^c = sum_i d_i^c on fluid sites (and
// -rho_ref^c, i.e. rho = 0, elsewhere), optionally with per-block FP64 partial
// sums of the fluid mass
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_density(DevParams P, const T *__restrict__ f,
                                                   const uint32_t *__restrict__ info, T *__restrict__ rho,
                                                   double *__restrict__ partial) {
    __shared__ double lds[2 * BLOCK];
    const long long n = (long long)blockIdx.x * BLOCK + threadIdx.x;
    double m[2] = {0.0, 0.0};
    if (n < P.N) {
        const bool fluid = site_class(info[n]) == CLS_FLUID;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            T dr = -(T)P.rho_ref[c];
            if (fluid) {
                dr = 0;
#pragma unroll
                for (int i = 0; i < Q; ++i) dr += f[(long long)(c * Q + i) * P.N + n];
                m[c] = (double)dr + P.rho_ref[c];
            }
            rho[c * P.N + n] = dr;
        }
    }
    if (partial) {
        block_sum<2>(m, lds);
        if (threadIdx.x == 0) {
            partial[2 * blockIdx.x + 0] = m[0];
            partial[2 * blockIdx.x + 1] = m[1];
        }
    }
}

// fixed-order sum of the per-block masses: M(t), baseline M(0), sentinel
__global__ void k_finalize_mass(const double *__restrict__ partial, int nb, DevState *st) {
    __shared__ double lds[2 * BLOCK];
    double m[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += BLOCK) {
        m[0] += partial[2 * b];
        m[1] += partial[2 * b + 1];
    }
    block_sum<2>(m, lds);
    if (threadIdx.x == 0) {
        st->Mstep[0] = m[0];
        st->Mstep[1] = m[1];
        if (!st->have_M0) {
            st->M0[0] = m[0];
            st->M0[1] = m[1];
            st->have_M0 = 1;
        }
        if (!isfinite(m[0]) || !isfinite(m[1])) st->unstable = 1;
    }
}

// ---------------------------------------------------------------------------
// virtual fluid (Sec. IV): on every shell site of particle p, rho^c is the mean
// of rho^c over its fluid 18-neighbours plus |colour| on the preferred
// component; written into the (deviation) density array in place.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_shell_fill(DevParams P, DevParticles D, const uint32_t *__restrict__ info,
                                                      T *__restrict__ rho) {
    const int p = blockIdx.x;
    const int cnt = min(D.shell_cnt[p], D.shell_cap[p]), off = D.shell_off[p];
    const double col = D.color[p];
    for (int k = threadIdx.x; k < cnt; k += BLOCK) {
        const long long s = D.shell[off + k];
        int x, y, z;
        site_xyz(s, P, x, y, z);
        T sum0 = 0, sum1 = 0;
        int nf = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const long long m = site_of(wrapc(x + cx(i), P.nx), wrapc(y + cy(i), P.ny), wrapc(z + cz(i), P.nz), P);
            if (site_class(info[m]) == CLS_FLUID) {
                sum0 += rho[m];
                sum1 += rho[P.N + m];
                ++nf;
            }
        }
        T r0 = nf ? sum0 / (T)nf : (T)0, r1 = nf ? sum1 / (T)nf : (T)0;
        if (col > 0.0) r0 += (T)fabs(col);
        if (col < 0.0) r1 += (T)fabs(col);
        rho[s] = r0;
        rho[P.N + s] = r1;
    }
}

// acc[c][a] = sum_{i=1..18} W_i Psi^c(x + c_i) c_ia from the density-deviation
// array, with Psi^c(x + c_i) - Psi^c(rho_ref) in place of Psi^c (same sum)
template <typename T>
__device__ __forceinline__ void neighbour_psi_sum(const T *__restrict__ rho, const DevParams &P, int x, int y, int z,
                                                  T acc[2][3]) {
    const T rho0 = (T)P.rho0;
    const T e[2] = {(T)P.psi_e[0], (T)P.psi_e[1]};
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[c][0] = acc[c][1] = acc[c][2] = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const long long m = site_of(wrapc(x + cx(i), P.nx), wrapc(y + cy(i), P.ny), wrapc(z + cz(i), P.nz), P);
        const T w = norm2(i) == 1 ? (T)P.w_face : (T)P.w_edge;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const T wp = w * psi_dev(rho[c * P.N + m], e[c], rho0);
            if (cx(i)) acc[c][0] += cx(i) > 0 ? wp : -wp;
            if (cy(i)) acc[c][1] += cy(i) > 0 ? wp : -wp;
            if (cz(i)) acc[c][2] += cz(i) > 0 ? wp : -wp;
        }
    }
}

// moments of one component from its stored values d_i = f_i - zeta_i rho_ref:
// dr = sum_i d_i, rho = dr + rho_ref, and j summed over opposite pairs (the
// reference part cancels exactly)
template <typename T>
__device__ __forceinline__ void moments(const T (&f)[Q], T ref, T &dr, T &r, T &jx, T &jy, T &jz) {
    dr = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) dr += f[i];
    r = dr + ref;
    jx = jy = jz = 0;
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const T d = f[i] - f[i + 1];
        if (cx(i)) jx += cx(i) > 0 ? d : -d;
        if (cy(i)) jy += cy(i) > 0 ? d : -d;
        if (cz(i)) jz += cz(i) > 0 ? d : -d;
    }
}

// equilibrium velocities of both components (Sec. II, Eq. (6))
template <typename T>
__device__ __forceinline__ void eq_velocity(const DevParams &P, const T r[2], const T j[2][3], const T F[2][3],
                                            T ueq[2][3]) {
    T ubar[3] = {0, 0, 0};
    if (P.velocity_mode == 0) {
        const T it0 = (T)(1.0 / P.tau[0]), it1 = (T)(1.0 / P.tau[1]);
        const T den = r[0] * it0 + r[1] * it1;
        if (den != (T)0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) ubar[a] = (j[0][a] * it0 + j[1][a] * it1) / den;
        }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const T tau = (T)P.tau[c];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            T base = ubar[a], shift = 0;
            if (r[c] != (T)0) {
                if (P.velocity_mode == 1) base = j[c][a] / r[c];
                shift = tau * F[c][a] / r[c];
            } else if (P.velocity_mode == 1) {
                base = 0;
            }
            ueq[c][a] = base + shift;
        }
    }
}

// ---------------------------------------------------------------------------
// collide and stream (two-pass variant, second sweep): reads f(t) at the
// site, densities of the neighbours from the density array, writes f(t+1).
// On shell sites it stores the Shan-Chen force for the particle sums.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_collide_stream(DevParams P, DevParticles D, const T *__restrict__ fin,
                                                          T *__restrict__ fout, const T *__restrict__ rho,
                                                          const uint32_t *__restrict__ info,
                                                          const int32_t *__restrict__ owner, T *__restrict__ fsc) {
    const long long n = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= P.N) return;
    const uint32_t inf = info[n];
    const uint32_t cls = site_class(inf);
    if (cls == CLS_SOLID || cls == CLS_WALL) return;
    int x, y, z;
    site_xyz(n, P, x, y, z);
    const T g = (T)P.g, rho0 = (T)P.rho0;
    T acc[2][3];
    neighbour_psi_sum(rho, P, x, y, z, acc);
    if (cls == CLS_SHELL) {
        const T ps0 = psi_of(rho[n] + (T)P.rho_ref[0], rho0), ps1 = psi_of(rho[P.N + n] + (T)P.rho_ref[1], rho0);
#pragma unroll
        for (int a = 0; a < 3; ++a) fsc[a * P.N + n] = -ps0 * g * acc[1][a] - ps1 * g * acc[0][a];
        return;
    }
    T f[2][Q];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i = 0; i < Q; ++i) f[c][i] = fin[(long long)(c * Q + i) * P.N + n];
    T dr[2], r[2], j[2][3], F[2][3];
#pragma unroll
    for (int c = 0; c < 2; ++c) moments(f[c], (T)P.rho_ref[c], dr[c], r[c], j[c][0], j[c][1], j[c][2]);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const T ps = psi_of(r[c], rho0);
#pragma unroll
        for (int a = 0; a < 3; ++a) F[c][a] = -ps * g * acc[1 - c][a] + r[c] * (T)P.body[a];
    }
    T ueq[2][3];
    eq_velocity(P, r, j, F, ueq);
    const int order = P.eq_order;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const T omega = (T)(1.0 / P.tau[c]);
        const T ux = ueq[c][0], uy = ueq[c][1], uz = ueq[c][2];
        const T u2 = ux * ux + uy * uy + uz * uz;
#pragma unroll
        for (int i = 0; i < Q; ++i)
            f[c][i] = f[c][i] - (f[c][i] - feq_dev_dir<T>(i, dr[c], r[c], ux, uy, uz, u2, order)) * omega;
    }
    // push: f*_i(x) -> f_i(x + c_i), or bounced back into f_opp(i)(x)
#pragma unroll
    for (int c = 0; c < 2; ++c) fout[(long long)(c * Q) * P.N + n] = f[c][0];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (inf & (1u << i)) {
            const long long m = site_of(wrapc(x + cx(i), P.nx), wrapc(y + cy(i), P.ny), wrapc(z + cz(i), P.nz), P);
            double ub[3], rb[3];
            solid_velocity(P, D, owner[m], x, y, z, i, ub, rb);
            const double cub = cx(i) * ub[0] + cy(i) * ub[1] + cz(i) * ub[2];
#pragma unroll
            for (int c = 0; c < 2; ++c)
                fout[(long long)(c * Q + opp(i)) * P.N + n] = f[c][i] - (T)(6.0 * zeta(i) * cub) * r[c];
        } else {
            const long long m = site_of(wrapc(x + cx(i), P.nx), wrapc(y + cy(i), P.ny), wrapc(z + cz(i), P.nz), P);
#pragma unroll
            for (int c = 0; c < 2; ++c) fout[(long long)(c * Q + i) * P.N + m] = f[c][i];
        }
    }
}

// ---------------------------------------------------------------------------
// fields of the current state (double): rho [2][N], j [2][N][3], F [2][N][3],
// u [N][3]; expects the density array filled (densities + virtual fluid)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_fields(DevParams P, const T *__restrict__ fin, const T *__restrict__ rho,
                                                  const uint32_t *__restrict__ info, double *__restrict__ out) {
    const long long n = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= P.N) return;
    const long long N = P.N;
    double *orho = out, *oj = out + 2 * N, *oF = out + 8 * N, *ou = out + 14 * N;
    const uint32_t cls = site_class(info[n]);
    for (int c = 0; c < 2; ++c) {
        orho[c * N + n] = 0.0;
        for (int a = 0; a < 3; ++a) {
            oj[(c * N + n) * 3 + a] = 0.0;
            oF[(c * N + n) * 3 + a] = 0.0;
        }
    }
    for (int a = 0; a < 3; ++a) ou[n * 3 + a] = 0.0;
    if (cls == CLS_SOLID || cls == CLS_WALL) return;
    int x, y, z;
    site_xyz(n, P, x, y, z);
    const T g = (T)P.g, rho0 = (T)P.rho0;
    T acc[2][3];
    neighbour_psi_sum(rho, P, x, y, z, acc);
    if (cls == CLS_SHELL) {
        const T ps0 = psi_of(rho[n] + (T)P.rho_ref[0], rho0), ps1 = psi_of(rho[N + n] + (T)P.rho_ref[1], rho0);
        for (int a = 0; a < 3; ++a) {
            oF[(0 * N + n) * 3 + a] = (double)(-ps0 * g * acc[1][a]);
            oF[(1 * N + n) * 3 + a] = (double)(-ps1 * g * acc[0][a]);
        }
        return;
    }
    T f[2][Q];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i = 0; i < Q; ++i) f[c][i] = fin[(long long)(c * Q + i) * N + n];
    T dr[2], r[2], j[2][3], F[2][3];
#pragma unroll
    for (int c = 0; c < 2; ++c) moments(f[c], (T)P.rho_ref[c], dr[c], r[c], j[c][0], j[c][1], j[c][2]);
    for (int c = 0; c < 2; ++c) {
        const T ps = psi_of(r[c], rho0);
        for (int a = 0; a < 3; ++a) F[c][a] = -ps * g * acc[1 - c][a] + r[c] * (T)P.body[a];
        orho[c * N + n] = (double)r[c];
        for (int a = 0; a < 3; ++a) {
            oj[(c * N + n) * 3 + a] = (double)j[c][a];
            oF[(c * N + n) * 3 + a] = (double)F[c][a];
        }
    }
    const double den = (double)r[0] + (double)r[1];
    for (int a = 0; a < 3; ++a) {
        const double num = (double)j[0][a] + 0.5 * (double)F[0][a] + (double)j[1][a] + 0.5 * (double)F[1][a];
        ou[n * 3 + a] = den != 0.0 ? num / den : 0.0;
    }
}

// per-block FP64 sums of mass [2] and momentum [3] over fluid sites
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_sums(DevParams P, const T *__restrict__ f, const uint32_t *__restrict__ info,
                                                double *__restrict__ partial) {
    __shared__ double lds[5 * BLOCK];
    const long long n = (long long)blockIdx.x * BLOCK + threadIdx.x;
    double v[5] = {0, 0, 0, 0, 0};
    if (n < P.N && site_class(info[n]) == CLS_FLUID) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            double m = P.rho_ref[c];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double di = (double)f[(long long)(c * Q + i) * P.N + n];
                m += di;
                v[2] += di * cx(i);
                v[3] += di * cy(i);
                v[4] += di * cz(i);
            }
            v[c] += m;
        }
    }
    block_sum<5>(v, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) partial[5 * blockIdx.x + k] = v[k];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblocks(long long n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

#define LB_DISPATCH(h, KERNEL_CALL_FLOAT, KERNEL_CALL_DOUBLE) \
    do {                                                     \
        if ((h)->prm.precision == LB_FP64) {                 \
            KERNEL_CALL_DOUBLE;                              \
        } else {                                             \
            KERNEL_CALL_FLOAT;                               \
        }                                                    \
    } while (0)

void launch_init_fluid(lb_handle *h) {
    const unsigned nb = nblocks(h->N);
    k_init_owner<<<nb, BLOCK, 0, h->stream>>>(h->dp, h->owner);
    LB_DISPATCH(h,
                (k_init_fluid<float><<<nb, BLOCK, 0, h->stream>>>(h->dp, h->prm.seed, h->prm.noise_amp, h->owner,
                                                                   (float *)h->f[h->cur])),
                (k_init_fluid<double><<<nb, BLOCK, 0, h->stream>>>(h->dp, h->prm.seed, h->prm.noise_amp, h->owner,
                                                                    (double *)h->f[h->cur])));
    k_info_dense<<<nb, BLOCK, 0, h->stream>>>(h->dp, h->owner, h->info);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_info_dense(lb_handle *h) {
    k_info_dense<<<nblocks(h->N), BLOCK, 0, h->stream>>>(h->dp, h->owner, h->info);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_owner_reset(lb_handle *h) {
    k_owner_reset<<<nblocks(h->N), BLOCK, 0, h->stream>>>(h->dp, h->owner);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_fill_int(lb_handle *h, int32_t *p, long long n, int32_t v) {
    if (n <= 0) return;
    k_fill_int<<<nblocks(n), BLOCK, 0, h->stream>>>(p, n, v);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_zero_solid(lb_handle *h, void *f) {
    const unsigned nb = nblocks(h->N);
    LB_DISPATCH(h, (k_zero_solid<float><<<nb, BLOCK, 0, h->stream>>>(h->dp, h->owner, (float *)f)),
                (k_zero_solid<double><<<nb, BLOCK, 0, h->stream>>>(h->dp, h->owner, (double *)f)));
    LB_HIP_CHECK(hipGetLastError());
}

void launch_density(lb_handle *h, const void *f, bool partial_sums) {
    const unsigned nb = nblocks(h->N);
    double *part = partial_sums ? h->partial : nullptr;
    LB_DISPATCH(h,
                (k_density<float><<<nb, BLOCK, 0, h->stream>>>(h->dp, (const float *)f, h->info, (float *)h->rho, part)),
                (k_density<double><<<nb, BLOCK, 0, h->stream>>>(h->dp, (const double *)f, h->info, (double *)h->rho,
                                                                 part)));
    LB_HIP_CHECK(hipGetLastError());
}

void launch_finalize_mass(lb_handle *h) {
    k_finalize_mass<<<1, BLOCK, 0, h->stream>>>(h->partial, (int)nblocks(h->N), h->dstate);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_shell_fill(lb_handle *h) {
    if (h->np == 0) return;
    LB_DISPATCH(h, (k_shell_fill<float><<<h->np, BLOCK, 0, h->stream>>>(h->dp, h->dpart, h->info, (float *)h->rho)),
                (k_shell_fill<double><<<h->np, BLOCK, 0, h->stream>>>(h->dp, h->dpart, h->info, (double *)h->rho)));
    LB_HIP_CHECK(hipGetLastError());
}

void launch_collide_stream(lb_handle *h, const void *fin, void *fout) {
    const unsigned nb = nblocks(h->N);
    LB_DISPATCH(h,
                (k_collide_stream<float><<<nb, BLOCK, 0, h->stream>>>(h->dp, h->dpart, (const float *)fin,
                                                                       (float *)fout, (const float *)h->rho, h->info,
                                                                       h->owner, (float *)h->fsc)),
                (k_collide_stream<double><<<nb, BLOCK, 0, h->stream>>>(h->dp, h->dpart, (const double *)fin,
                                                                        (double *)fout, (const double *)h->rho, h->info,
                                                                        h->owner, (double *)h->fsc)));
    LB_HIP_CHECK(hipGetLastError());
}

void launch_fields(lb_handle *h, const void *f, double *out) {
    const unsigned nb = nblocks(h->N);
    LB_DISPATCH(h,
                (k_fields<float><<<nb, BLOCK, 0, h->stream>>>(h->dp, (const float *)f, (const float *)h->rho, h->info,
                                                               out)),
                (k_fields<double><<<nb, BLOCK, 0, h->stream>>>(h->dp, (const double *)f, (const double *)h->rho,
                                                                h->info, out)));
    LB_HIP_CHECK(hipGetLastError());
}

void launch_sums(lb_handle *h, const void *f) {
    const unsigned nb = nblocks(h->N);
    LB_DISPATCH(h, (k_sums<float><<<nb, BLOCK, 0, h->stream>>>(h->dp, (const float *)f, h->info, h->partial)),
                (k_sums<double><<<nb, BLOCK, 0, h->stream>>>(h->dp, (const double *)f, h->info, h->partial)));
    LB_HIP_CHECK(hipGetLastError());
}

}  // namespace lbm
