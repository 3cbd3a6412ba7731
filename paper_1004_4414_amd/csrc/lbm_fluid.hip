// Fluid kernels for gfx950: initial state, densities, virtual fluid,
// Shan-Chen force, BGK collision with the velocity shift and pull streaming
// (Secs. II-IV of Jansen & Harting), bounce-back at the walls, plus the field
// and sum kernels behind the observables.
//
// Storage: populations in storage blocks of 64 consecutive sites (site index
// n = (z*ny + y)*nx + x), both components of a direction side by side, so a
// wavefront's 64 lanes read or write one aligned 512-byte run per direction;
// slot (i, z) holds what site z + c_i receives in direction i (lbm_device.h).
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
    unsigned n;
    int x, y, z;
    if (!dense_site(P, n, x, y, z)) return;
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
// stored as f - zeta_i rho_ref^c in the slots (i, x - c_i) the site reads
template <typename S>
__global__ void k_init_fluid(DevParams P, uint64_t seed, double noise, const int32_t *__restrict__ owner,
                             S *__restrict__ f) {
#pragma clang fp contract(off)
    using T = Cmp<S>;
    unsigned n;
    int x, y, z;
    if (!dense_site(P, n, x, y, z)) return;
    if (owner[n] != OWN_FLUID) return;
    const NbrOffsets o(P, x, y, z);
    double r[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const double U = (double)(splitmix64_at(seed, 2ull * (unsigned long long)n + c) >> 11) *
                         (1.0 / 9007199254740992.0);
        r[c] = P.rho_init[c] + noise * (2.0 * U - 1.0);
    }
    Unroll<Q>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const unsigned dst = i == 0 ? n : (unsigned)((int)n + o.template off<opp(i)>());
        store_pop(f, pidx(0, i, dst), (T)(zeta(i) * r[0] - zeta(i) * P.rho_ref[0]),
                  (T)(zeta(i) * r[1] - zeta(i) * P.rho_ref[1]));
    });
}

__global__ void k_info_dense(DevParams P, const int32_t *__restrict__ owner, uint32_t *__restrict__ info) {
    unsigned n;
    int x, y, z;
    if (!dense_site(P, n, x, y, z)) return;
    info[n] = compute_info(n, P, owner);
}

__global__ void k_owner_reset(DevParams P, int32_t *owner) {
    unsigned n;
    int x, y, z;
    if (!dense_site(P, n, x, y, z)) return;
    if (owner[n] >= 0) owner[n] = OWN_FLUID;
}

__global__ void k_clear_flags(uint32_t *info, long long n) {
    const long long k = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (k < n) info[k] &= ~INFO_FLAG;
}

__global__ void k_fill_int(int32_t *p, long long n, int32_t v) {
    const long long k = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (k < n) p[k] = v;
}

// ---------------------------------------------------------------------------
// density deviations rho^c - rho_ref^c = sum_i d_i^c and Psi^c - Psi^c(rho_ref)
// on fluid sites (rho = 0 elsewhere), optionally with per-wavefront FP64
// partial sums of the fluid mass (a shuffle tree, no barrier, so no
// wavefront waits for the others of its block)
// ---------------------------------------------------------------------------
// ROWS: row-aligned addressing (nx a multiple of 64)
// Bounced populations formed by the density sweep (sweep_bounce in
// lbm_api.hip): the link kernel of the previous step left the solid sites'
// slots of the links of fluid site n unwritten; the density sweep puts in
// place of each such pull the pair formed from n's own slot (i, n), n's
// density deviations of that step (rho_prev) and the sphere state of the
// bounce, bitwise the value the link kernel would have written, and stores
// it into the slot it has just pulled, for the collide sweep.  A flagged
// class word marks a site whose links the map update wrote out.
template <typename S, typename T>
__device__ __forceinline__ bool sweep_bounces_here(const DevParams &P, uint32_t inf) {
    return P.redirect && site_class(inf) == CLS_FLUID && !(inf & INFO_FLAG) && (inf & 0x7fffeu);
}
template <typename S, typename T>
__device__ __forceinline__ void sweep_bounce_put(const DevParams &P, const DevParticles &D, S *f,
                                                 const T *__restrict__ rho_prev, const int32_t *__restrict__ owner,
                                                 unsigned n, int x, int y, int z, uint32_t inf, T (&fv)[2][Q]) {
    const uint32_t bits = inf & 0x7fffeu;
    // every load at once: the site's own slots of its link directions (other
    // lanes of the instruction read slot 0), its densities of the bounce's
    // step and the sphere of its first link (of every link when they belong
    // to several spheres)
    Pair<T> raw[Q - 1];
    Unroll<Q - 1>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value + 1;
        raw[i - 1] = load_pop(f, pidx(0, ((bits >> i) & 1u) ? i : 0, n));
    });
    const Pair<T> dr = load_pair(rho_prev, sidx(0, n));
    const int i0 = __ffs(bits) - 1;
    const int32_t q0 =
        owner[site_of(wrapc(x + cx(i0), P.nx), wrapc(y + cy(i0), P.ny), wrapc(z + cz(i0), P.nz), P)];
    double u[3] = {0.0, 0.0, 0.0};
    if (q0 >= 0) {  // a sphere (lattices with spheres have no walls)
        double R[3], U[3], W[3];
        for (int a = 0; a < 3; ++a) {
            R[a] = D.Rl[3 * q0 + a];
            U[a] = D.Ul[3 * q0 + a];
            W[a] = D.Wl[3 * q0 + a];
        }
        rigid_u(P, R, U, W, x, y, z, u);
    }
    const bool multi = (inf & INFO_MULTI) != 0u;
    Unroll<Q - 1>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value + 1;
        if ((bits >> i) & 1u) {
            const long long sn = site_of(wrapc(x + cx(i), P.nx), wrapc(y + cy(i), P.ny), wrapc(z + cz(i), P.nz), P);
            double ui[3] = {u[0], u[1], u[2]};
            int32_t q = q0;
            if (multi) {
                q = owner[sn];
                if (q >= 0 && q != q0) {
                    double R[3], U[3], W[3];
                    for (int a = 0; a < 3; ++a) {
                        R[a] = D.Rl[3 * q + a];
                        U[a] = D.Ul[3 * q + a];
                        W[a] = D.Wl[3 * q + a];
                    }
                    rigid_u(P, R, U, W, x, y, z, ui);
                }
            }
            if (q >= 0) {
                T b0, b1, w0, w1;
                bounce_pair<T>(P, cu_dot(i, ui), i, raw[i - 1].x, raw[i - 1].y, dr.x, dr.y, b0, b1, w0, w1);
                fv[0][opp(i)] = Storage<S>::rt(b0);  // as stored and loaded back
                fv[1][opp(i)] = Storage<S>::rt(b1);
                // into the slot this thread has just pulled (its one reader),
                // a line the caches still hold: the collide sweep pulls it
                store_pop_keep(f, pidx(0, opp(i), (unsigned)sn), b0, b1);
            }
        }
    });
}

// (the populations are not restrict-qualified where the sweep stores into them)
template <typename S, bool BOUNCE>
using DensityPops = typename std::conditional<BOUNCE, const S *, const S *__restrict__>::type;
template <typename S, bool ROWS, bool BOUNCE = false, typename T = Cmp<S>>
__device__ __forceinline__ void density_body(const DevParams &P, DensityPops<S, BOUNCE> f,
                                             const uint32_t *__restrict__ info, T *__restrict__ rho,
                                             T *__restrict__ psi, double *__restrict__ partial, const Grid &g,
                                             const DevParticles &D, const int32_t *__restrict__ owner,
                                             const T *__restrict__ rho_prev) {
    double m[2] = {0.0, 0.0};
    unsigned n;
    int x, y, z;
    if (ROWS ? dense_site_rows(P, g, n, x, y, z) : dense_site(P, g, n, x, y, z)) {
        // the pulls are issued before the class word arrives (every address is
        // in the lattice); non-fluid sites discard the sum
        T s0 = 0, s1 = 0;  // in direction order, as every density sum of the step
        uint32_t inf;
        if constexpr (BOUNCE) {
            T fv[2][Q];
            if constexpr (ROWS) {
                const RowView<S> rv(P, x, y, z);
                pull_load_rows(f, rv, fv);
            } else {
                const NbrOffsets o(P, x, y, z);
                pull_load(f, n, o, fv);
            }
            inf = __builtin_nontemporal_load(info + n);
            if (sweep_bounces_here<S, T>(P, inf))
                sweep_bounce_put<S, T>(P, D, const_cast<S *>(f), rho_prev, owner, n, x, y, z, inf, fv);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                s0 += fv[0][i];
                s1 += fv[1][i];
            }
        } else {
            if constexpr (ROWS) {
                const RowView<S> rv(P, x, y, z);
                pull_sum_rows(f, rv, s0, s1);
            } else {
                const NbrOffsets o(P, x, y, z);
                pull_sum(f, n, o, s0, s1);
            }
            // the class word is read once per sweep: streamed like the pulls
            inf = __builtin_nontemporal_load(info + n);
        }
        const bool fluid = site_class(inf) == CLS_FLUID;
        const T irho0 = (T)P.inv_rho0;
        T dr[2] = {-(T)P.rho_ref[0], -(T)P.rho_ref[1]};
        if (fluid) {
            dr[0] = s0;
            dr[1] = s1;
            m[0] = (double)dr[0] + P.rho_ref[0];
            m[1] = (double)dr[1] + P.rho_ref[1];
        }
        // read back by the collide sweep, after the rest of this sweep
        store_pair_stream(rho, sidx(0, n), dr[0], dr[1]);
        store_pair_stream(psi, sidx(0, n), psi_dev(dr[0], (T)P.psi_e[0], irho0),
                          psi_dev(dr[1], (T)P.psi_e[1], irho0));
    }
    if (partial) {
#pragma unroll
        for (int c = 0; c < 2; ++c)
            for (int off = 32; off > 0; off >>= 1) m[c] += __shfl_down(m[c], off, 64);
        if ((threadIdx.x & 63) == 0) {
            const unsigned w = g.bid * (BLOCK / 64) + (threadIdx.x >> 6);
            partial[2 * w + 0] = m[0];
            partial[2 * w + 1] = m[1];
        }
    }
}
template <typename S, bool ROWS, typename T = Cmp<S>>
__global__ __launch_bounds__(BLOCK) void k_density(DevParams P, const S *__restrict__ f,
                                                   const uint32_t *__restrict__ info, T *__restrict__ rho,
                                                   T *__restrict__ psi, double *__restrict__ partial) {
    density_body<S, ROWS, false>(P, f, info, rho, psi, partial, own_grid(), DevParticles{}, nullptr,
                                 (const T *)nullptr);
}
// the variant that forms the pending bounced populations (it stores into f)
template <typename S, bool ROWS, typename T = Cmp<S>>
__global__ __launch_bounds__(BLOCK) void k_density_bounce(DevParams P, S *f, const uint32_t *__restrict__ info,
                                                          T *__restrict__ rho, T *__restrict__ psi,
                                                          double *__restrict__ partial, DevParticles D,
                                                          const int32_t *__restrict__ owner,
                                                          const T *__restrict__ rho_prev) {
    density_body<S, ROWS, true>(P, f, info, rho, psi, partial, own_grid(), D, owner, rho_prev);
}

// fixed-order sum of the per-block masses: M(t), baseline M(0), sentinel.
// fin_blocks(nb) blocks (one per FIN_PER_BLOCK partials, at most FIN_BLOCKS)
// each sum a contiguous range of the partials (8 independent sums per thread,
// then a fixed tree); the last block to finish (an integer counter) sums their
// results in block order and resets the counter, so the total does not
// depend on which block finishes last.  Blocks past fin_blocks(nb) return.
constexpr int FIN_THREADS = 256;
static_assert(FIN_BLOCKS <= FIN_THREADS, "the last block sums one block result per thread");
__device__ __forceinline__ void finalize_body(const double *__restrict__ partial, int nb, DevState *st,
                                              unsigned bid) {
    __shared__ double lds[2][FIN_THREADS];
    __shared__ int last;
    const int t = threadIdx.x;
    const int nf = fin_blocks(nb);
    if ((int)bid >= nf) return;  // uniform over the block
    const int chunk = (nb + nf - 1) / nf;
    const int b_lo = (int)bid * chunk, b_hi = min(nb, b_lo + chunk);
    double a[2][8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[0][j] = a[1][j] = 0.0;
    for (int b0 = b_lo + t; b0 < b_hi; b0 += 8 * FIN_THREADS) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int b = b0 + j * FIN_THREADS;
            if (b < b_hi) {
                a[0][j] += partial[2 * b];
                a[1][j] += partial[2 * b + 1];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
        lds[c][t] = ((a[c][0] + a[c][1]) + (a[c][2] + a[c][3])) + ((a[c][4] + a[c][5]) + (a[c][6] + a[c][7]));
    __syncthreads();
    for (int s = FIN_THREADS / 2; s > 0; s >>= 1) {
        if (t < s) {
            lds[0][t] += lds[0][t + s];
            lds[1][t] += lds[1][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        st->fin_part[2 * bid] = lds[0][0];
        st->fin_part[2 * bid + 1] = lds[1][0];
        __threadfence();
        last = atomicAdd(&st->fin_count, 1u) == (unsigned)nf - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    const volatile double *fp = st->fin_part;
    for (int c = 0; c < 2; ++c) lds[c][t] = t < nf ? fp[2 * t + c] : 0.0;
    __syncthreads();
    for (int s = FIN_BLOCKS / 2; s > 0; s >>= 1) {
        if (t < s) {
            lds[0][t] += lds[0][t + s];
            lds[1][t] += lds[1][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        const double m0 = lds[0][0], m1 = lds[1][0];
        st->Mstep[0] = m0;
        st->Mstep[1] = m1;
        if (!st->have_M0) {
            st->M0[0] = m0;
            st->M0[1] = m1;
            st->have_M0 = 1;
        }
        if (!isfinite(m0) || !isfinite(m1)) st->unstable = 1;
        st->fin_count = 0;
    }
}
__global__ __launch_bounds__(FIN_THREADS) void k_finalize_mass(const double *__restrict__ partial, int nb,
                                                               DevState *st) {
    finalize_body(partial, nb, st, blockIdx.x);
}

// ---------------------------------------------------------------------------
// virtual fluid (Sec. IV): on every shell site of particle p, rho^c is the mean
// of rho^c over its fluid 18-neighbours plus |colour| on the preferred
// component; only its Psi - Psi(rho_ref) is stored (in the Psi array), since
// every later use of a shell site's density goes through Psi.
// ---------------------------------------------------------------------------
// A virtual-fluid site per thread; the single-lattice launch gives each
// sphere one block per SHELL_THREADS sites of its list capacity (chunk c takes
// sites c * SHELL_THREADS + t, blocks past the list end return at once), the
// batch launch one block per sphere (nchunk = 1)
constexpr int SHELL_THREADS = 256;
template <typename T>
__device__ __forceinline__ void shell_fill_body(const DevParams &P, const DevParticles &D,
                                                const uint32_t *__restrict__ info, T *__restrict__ rho,
                                                T *__restrict__ psi, int p, int chunk, int nchunk) {
    const int cnt = min(D.shell_cnt[p], D.shell_cap[p]), off = D.shell_off[p];
    if (chunk * SHELL_THREADS >= cnt) return;  // uniform over the block
    const double col = D.color[p];
    const T irho0 = (T)P.inv_rho0;
    for (int k = chunk * SHELL_THREADS + threadIdx.x; k < cnt; k += nchunk * SHELL_THREADS) {
        const long long s = D.shell[off + k];
        int x, y, z;
        site_xyz(s, P, x, y, z);
        // the class word of a shell site flags its non-fluid neighbours; every
        // neighbour's density is loaded (the addresses are in the box) and
        // masked afterwards, so the loads of a site are in flight together
        const uint32_t inf = info[s];
        T sum0 = 0, sum1 = 0;
        int nf = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const unsigned m =
                (unsigned)site_of(wrapc(x + cx(i), P.nx), wrapc(y + cy(i), P.ny), wrapc(z + cz(i), P.nz), P);
            const bool fl = !((inf >> i) & 1u);
            const Pair<T> a = load_pair(rho, sidx(0, m));
            const T a0 = a.x, a1 = a.y;
            sum0 += fl ? a0 : (T)0;
            sum1 += fl ? a1 : (T)0;
            nf += fl;
        }
        T r0 = nf ? sum0 / (T)nf : (T)0, r1 = nf ? sum1 / (T)nf : (T)0;
        if (col > 0.0) r0 += (T)fabs(col);
        if (col < 0.0) r1 += (T)fabs(col);
        store_pair(psi, sidx(0, (unsigned)s), psi_dev(r0, (T)P.psi_e[0], irho0), psi_dev(r1, (T)P.psi_e[1], irho0));
    }
}
template <typename T>
__global__ __launch_bounds__(SHELL_THREADS) void k_shell_fill(DevParams P, DevParticles D,
                                                              const uint32_t *__restrict__ info, T *__restrict__ rho,
                                                              T *__restrict__ psi, int nchunk) {
    // chunk-major: the first chunks of every sphere are dispatched first
    const int np = (int)(gridDim.x / (unsigned)nchunk);
    shell_fill_body(P, D, info, rho, psi, (int)(blockIdx.x % (unsigned)np), (int)(blockIdx.x / (unsigned)np), nchunk);
}

// Psi^c(x + c_i) - Psi^c(rho_ref) of the 18 neighbours (pn[c][i-1]) and of
// the site itself (own[c]; on a virtual-fluid site it gives the site's Psi
// without a second round trip to memory)
template <typename T>
__device__ __forceinline__ void load_psi_neighbours(const T *__restrict__ psi, unsigned n, const NbrOffsets &o,
                                                    T (&pn)[2][Q - 1], T (&own)[2]) {
    const Pair<T> v0 = load_pair(psi, sidx(0, n));
    own[0] = v0.x;
    own[1] = v0.y;
    Unroll<Q - 1>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value + 1;
        const unsigned m = (unsigned)((int)n + o.template off<i>());
        const Pair<T> v = load_pair(psi, sidx(0, m));
        pn[0][i - 1] = v.x;
        pn[1][i - 1] = v.y;
    });
}

// the same with row-aligned addressing
template <typename S, typename T = Cmp<S>>
__device__ __forceinline__ void load_psi_neighbours_rows(const T *__restrict__ psi, const RowView<S> &rv,
                                                         T (&pn)[2][Q - 1], T (&own)[2]) {
    const char *base = reinterpret_cast<const char *>(psi);
    const Pair<T> v0 = *reinterpret_cast<const Pair<T> *>(base + rv.row(0, 0) * rv.frow + rv.fo[1]);
    own[0] = v0.x;
    own[1] = v0.y;
    Unroll<Q - 1>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value + 1;
        const char *row = base + rv.row(cy(i), cz(i)) * rv.frow;
        const Pair<T> v = *reinterpret_cast<const Pair<T> *>(row + rv.fo[1 + cx(i)]);
        pn[0][i - 1] = v.x;
        pn[1][i - 1] = v.y;
    });
}

// ---------------------------------------------------------------------------
// collide and stream (two-pass variant, second sweep): populations of the
// site, Psi of the neighbours from the Psi array.  On shell sites it stores
// the Shan-Chen force for the particle sums.  Every load of a site is issued
// before its classification is known (all addresses lie in the box), so a
// wavefront has its whole working set in flight at once.  Every site stores
// its 19 own slots (f* on fluid sites, zeros elsewhere) with the wavefront's
// full lane mask; ROWS selects row-aligned addressing (nx a multiple of 64).
// ---------------------------------------------------------------------------
template <typename S, typename M, bool ROWS, typename T = Cmp<S>>
__device__ __forceinline__ void collide_body(const DevParams &P, const S *__restrict__ fin, S *__restrict__ fout,
                                             const T *__restrict__ psi, const uint32_t *__restrict__ info,
                                             T *__restrict__ fsc, const Grid &g) {
    unsigned n;
    int x, y, z;
    if (!(ROWS ? dense_site_rows(P, g, n, x, y, z) : dense_site(P, g, n, x, y, z))) return;
    T f[2][Q];
    T pn[2][Q - 1], own_psi[2];
    if constexpr (ROWS) {
        const RowView<S> rv(P, x, y, z);
        pull_load_rows(fin, rv, f);
        load_psi_neighbours_rows(psi, rv, pn, own_psi);
    } else {
        const NbrOffsets o(P, x, y, z);
        pull_load(fin, n, o, f);
        load_psi_neighbours(psi, n, o, pn, own_psi);
    }
    const uint32_t inf = __builtin_nontemporal_load(info + n);  // read once per sweep
    hold_loads(f[0]);
    hold_loads(f[1]);
    hold_loads(pn[0]);
    hold_loads(pn[1]);
    hold_loads(own_psi);
    const uint32_t cls = site_class(inf);
    T F[3] = {0, 0, 0};
    if (cls == CLS_FLUID || cls == CLS_SHELL) {
        T acc[2][3];
        psi_force_sum(P, pn, acc);
        if (cls == CLS_SHELL) {
            shell_force(P, own_psi, acc, F);
        } else {
            double m0 = 0.0, m1 = 0.0;
            collide_site<M>(P, f, acc, inf, n, (T *)nullptr, m0, m1);
        }
    }
    if (cls != CLS_FLUID) {
#pragma unroll
        for (int i = 0; i < Q; ++i) f[0][i] = f[1][i] = (T)0;
    }
    if (cls == CLS_SHELL) {
        if (shell_force_in_slots<S>(inf)) {
            put_shell_force(f, F, inf);
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) fsc[vidx(a, n)] = F[a];
        }
    }
    if constexpr (ROWS) {
        const RowView<S> rv(P, x, y, z);
        char *own = reinterpret_cast<char *>(fout) + rv.row(0, 0) * rv.prow + rv.po[1];
        Unroll<Q>::run([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            store_pop(reinterpret_cast<S *>(own + (size_t)i * RowView<S>::DB), 0, f[0][i], f[1][i]);
        });
    } else {
        Unroll<Q>::run([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            store_pop(fout, pidx(0, i, n), f[0][i], f[1][i]);
        });
    }
}
template <typename S, typename M, bool ROWS, typename T = Cmp<S>>
__global__ __launch_bounds__(BLOCK) LBM_COLLIDE_ATTR void k_collide_stream(DevParams P, const S *__restrict__ fin,
                                                                          S *__restrict__ fout,
                                                                          const T *__restrict__ psi,
                                                                          const uint32_t *__restrict__ info,
                                                                          T *__restrict__ fsc) {
    collide_body<S, M, ROWS>(P, fin, fout, psi, info, fsc, own_grid());
}

// ---------------------------------------------------------------------------
// bounce-back at the two walls, Eq. (16): for a fluid site x next to a wall
// and a direction i with x + c_i in the wall, f*_i(x) (slot (i, x), written by
// the sweep) is reflected into slot (opp(i), x + c_i) less the moving-wall
// term 6 zeta_i rho^c(x) (c_i . u_wall).  Only the planes next to the walls
// hold such links; the grid covers both (one thread per site of the two
// planes).
// ---------------------------------------------------------------------------
template <typename S, typename T = Cmp<S>>
__global__ __launch_bounds__(BLOCK) void k_wall_links(DevParams P, S *__restrict__ fout, const T *__restrict__ rho,
                                                      const uint32_t *__restrict__ info,
                                                      const int32_t *__restrict__ owner) {
    const int ax = P.wall_axis;
    const int L = ax == 0 ? P.nx : (ax == 1 ? P.ny : P.nz);
    const int ua = ax == 0 ? P.ny : P.nx;  // the two in-plane axes, u fastest
    const int va = ax == 2 ? P.ny : P.nz;
    const long long plane = (long long)ua * va;
    const long long k = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= 2 * plane) return;
    const int pos = k < plane ? 1 : L - 2;
    if (k >= plane && L - 2 == 1) return;  // one plane touches both walls
    const int u = (int)((k % plane) % ua), v = (int)((k % plane) / ua);
    const int x = ax == 0 ? pos : u, y = ax == 1 ? pos : (ax == 0 ? u : v), z = ax == 2 ? pos : v;
    const unsigned n = (unsigned)(((long long)z * P.ny + y) * P.nx + x);
    const uint32_t inf = info[n];
    if (site_class(inf) != CLS_FLUID) return;
    uint32_t bits = inf & 0x7fffeu;
    while (bits) {
        const int i = __ffs(bits) - 1;
        bits &= bits - 1;
        const int xn = wrapc(x + cx(i), P.nx), yn = wrapc(y + cy(i), P.ny), zn = wrapc(z + cz(i), P.nz);
        const unsigned m = (unsigned)(((long long)zn * P.ny + yn) * P.nx + xn);
        const int32_t own = owner[m];
        if (own != OWN_WALL_LO && own != OWN_WALL_HI) continue;
        const bool lo = own == OWN_WALL_LO;
        double cub = 0.0;
        if (cx(i)) cub += cx(i) * (lo ? P.wall_vel[0][0] : P.wall_vel[1][0]);
        if (cy(i)) cub += cy(i) * (lo ? P.wall_vel[0][1] : P.wall_vel[1][1]);
        if (cz(i)) cub += cz(i) * (lo ? P.wall_vel[0][2] : P.wall_vel[1][2]);
        const Pair<T> ff = load_pop(fout, pidx(0, i, n));  // f*_i(x), stored by the sweep in slot (i, x)
        if (cub == 0.0) {
            store_pop(fout, pidx(0, opp(i), m), ff.x, ff.y);
            continue;
        }
        const T wz = (T)(6.0 * zeta(i) * cub);
        const Pair<T> rr = load_pair(rho, sidx(0, n));
        store_pop(fout, pidx(0, opp(i), m), ff.x - wz * (rr.x + (T)P.rho_ref[0]), ff.y - wz * (rr.y + (T)P.rho_ref[1]));
    }
}

// ---------------------------------------------------------------------------
// fields of the current state (double): rho [2][N], j [2][N][3], F [2][N][3],
// u [N][3]; expects the density and Psi arrays filled (with virtual fluid)
// ---------------------------------------------------------------------------
template <typename S, typename T = Cmp<S>>
__global__ __launch_bounds__(BLOCK) void k_fields(DevParams P, const S *__restrict__ fin, const T *__restrict__ rho,
                                                  const T *__restrict__ psi, const uint32_t *__restrict__ info,
                                                  double *__restrict__ out) {
    unsigned n;
    int x, y, z;
    if (!dense_site(P, n, x, y, z)) return;
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
    const NbrOffsets o(P, x, y, z);
    const T g = (T)P.g, rho0 = (T)P.rho0, irho0 = (T)P.inv_rho0;
    T acc[2][3], pn[2][Q - 1], own_psi[2];
    load_psi_neighbours(psi, n, o, pn, own_psi);
    psi_force_sum(P, pn, acc);
    if (cls == CLS_SHELL) {  // Psi of the site: its stored deviation plus Psi(rho_ref) = rho0 - psi_e
        const T ps0 = own_psi[0] + (T)(P.rho0 - P.psi_e[0]);
        const T ps1 = own_psi[1] + (T)(P.rho0 - P.psi_e[1]);
        for (int a = 0; a < 3; ++a) {
            oF[(0 * N + n) * 3 + a] = (double)(-ps0 * g * acc[1][a]);
            oF[(1 * N + n) * 3 + a] = (double)(-ps1 * g * acc[0][a]);
        }
        return;
    }
    T f[2][Q];
    pull_load(fin, n, o, f);
    T dr[2], r[2], j[2][3], F[2][3];
#pragma unroll
    for (int c = 0; c < 2; ++c) moments(f[c], (T)P.rho_ref[c], dr[c], r[c], j[c][0], j[c][1], j[c][2]);
    for (int c = 0; c < 2; ++c) {
        const T ps = psi_of(r[c], rho0, irho0);
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
template <typename S, typename T = Cmp<S>>
__global__ __launch_bounds__(BLOCK) void k_sums(DevParams P, const S *__restrict__ fin,
                                                const uint32_t *__restrict__ info, double *__restrict__ partial) {
    __shared__ double lds[5 * (BLOCK / 64)];
    double v[5] = {0, 0, 0, 0, 0};
    unsigned n;
    int x, y, z;
    if (dense_site(P, n, x, y, z)) {
        if (site_class(info[n]) == CLS_FLUID) {
            T f[2][Q];
            pull_load(fin, n, NbrOffsets(P, x, y, z), f);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                double m = P.rho_ref[c];
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const double di = (double)f[c][i];
                    m += di;
                    v[2] += di * cx(i);
                    v[3] += di * cy(i);
                    v[4] += di * cz(i);
                }
                v[c] += m;
            }
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
static inline unsigned dense_blocks(const lb_handle *h) { return nblocks(h->N); }

void launch_init_fluid(lb_handle *h) {
    const unsigned nb = dense_blocks(h);
    k_init_owner<<<nb, BLOCK, 0, h->stream>>>(h->dp, h->owner);
    with_storage(h->prm, [&](auto tag) {
        using S = typename decltype(tag)::type;
        k_init_fluid<S><<<nb, BLOCK, 0, h->stream>>>(h->dp, h->prm.seed, h->prm.noise_amp, h->owner, (S *)h->f[h->cur]);
    });
    k_info_dense<<<nb, BLOCK, 0, h->stream>>>(h->dp, h->owner, h->info);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_info_dense(lb_handle *h) {
    k_info_dense<<<dense_blocks(h), BLOCK, 0, h->stream>>>(h->dp, h->owner, h->info);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_owner_reset(lb_handle *h) {
    k_owner_reset<<<dense_blocks(h), BLOCK, 0, h->stream>>>(h->dp, h->owner);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_fill_int(lb_handle *h, int32_t *p, long long n, int32_t v) {
    if (n <= 0) return;
    k_fill_int<<<nblocks(n), BLOCK, 0, h->stream>>>(p, n, v);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_clear_flags(lb_handle *h) {
    k_clear_flags<<<nblocks(h->N), BLOCK, 0, h->stream>>>(h->info, h->N);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_density(lb_handle *h, const void *f, bool partial_sums) {
    const unsigned nb = dense_blocks(h);
    double *part = partial_sums ? h->partial : nullptr;
    with_storage(h->prm, [&](auto tag) {
        using S = typename decltype(tag)::type;
        using T = Cmp<S>;
        const bool rows = h->prm.nx % (int)VB == 0;
        if (h->dp.redirect) {
            const T *rp = (const T *)h->rho_prev;
            if (rows)
                k_density_bounce<S, true><<<nb, BLOCK, 0, h->stream>>>(h->dp, (S *)f, h->info, (T *)h->rho,
                                                                       (T *)h->psi, part, h->dpart, h->owner, rp);
            else
                k_density_bounce<S, false><<<nb, BLOCK, 0, h->stream>>>(h->dp, (S *)f, h->info, (T *)h->rho,
                                                                        (T *)h->psi, part, h->dpart, h->owner, rp);
        } else if (rows) {
            k_density<S, true><<<nb, BLOCK, 0, h->stream>>>(h->dp, (const S *)f, h->info, (T *)h->rho, (T *)h->psi,
                                                            part);
        } else {
            k_density<S, false><<<nb, BLOCK, 0, h->stream>>>(h->dp, (const S *)f, h->info, (T *)h->rho, (T *)h->psi,
                                                             part);
        }
    });
    LB_HIP_CHECK(hipGetLastError());
}

// the density pass leaves one partial mass per wavefront
void launch_finalize_mass(lb_handle *h) { launch_finalize_mass_n(h, (int)dense_blocks(h) * (BLOCK / 64)); }

void launch_finalize_mass_n(lb_handle *h, int nb) {
    k_finalize_mass<<<fin_blocks(nb), FIN_THREADS, 0, h->stream>>>(h->partial, nb, h->dstate);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_shell_fill(lb_handle *h) {
    if (h->np == 0) return;
    const int nchunk = std::max(1, (h->max_shell_cap + SHELL_THREADS - 1) / SHELL_THREADS);
    const unsigned nb = (unsigned)h->np * (unsigned)nchunk;
    if (h->prm.precision == LB_FP64)
        k_shell_fill<double><<<nb, SHELL_THREADS, 0, h->stream>>>(h->dp, h->dpart, h->info, (double *)h->rho,
                                                                  (double *)h->psi, nchunk);
    else
        k_shell_fill<float><<<nb, SHELL_THREADS, 0, h->stream>>>(h->dp, h->dpart, h->info, (float *)h->rho,
                                                                 (float *)h->psi, nchunk);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_collide_stream(lb_handle *h, const void *fin, void *fout) {
    const unsigned nb = dense_blocks(h);
    const bool rows = h->prm.nx % (int)VB == 0;
    with_storage(h->prm, [&](auto tag) {
        using S = typename decltype(tag)::type;
        using T = Cmp<S>;
        with_model(h->prm, [&](auto m) {
            if (rows)
                k_collide_stream<S, decltype(m), true><<<nb, BLOCK, 0, h->stream>>>(
                    h->dp, (const S *)fin, (S *)fout, (const T *)h->psi, h->info, (T *)h->fsc);
            else
                k_collide_stream<S, decltype(m), false><<<nb, BLOCK, 0, h->stream>>>(
                    h->dp, (const S *)fin, (S *)fout, (const T *)h->psi, h->info, (T *)h->fsc);
        });
    });
    LB_HIP_CHECK(hipGetLastError());
}

void launch_wall_links(lb_handle *h, void *fout) {
    const int ax = h->prm.wall_axis;
    if (ax < 0) return;
    const long long plane = ax == 0 ? (long long)h->prm.ny * h->prm.nz
                                    : (ax == 1 ? (long long)h->prm.nx * h->prm.nz : (long long)h->prm.nx * h->prm.ny);
    const unsigned nb = nblocks(2 * plane);
    with_storage(h->prm, [&](auto tag) {
        using S = typename decltype(tag)::type;
        using T = Cmp<S>;
        k_wall_links<S><<<nb, BLOCK, 0, h->stream>>>(h->dp, (S *)fout, (const T *)h->rho, h->info, h->owner);
    });
    LB_HIP_CHECK(hipGetLastError());
}

void launch_fields(lb_handle *h, const void *f, double *out) {
    const unsigned nb = dense_blocks(h);
    with_storage(h->prm, [&](auto tag) {
        using S = typename decltype(tag)::type;
        using T = Cmp<S>;
        k_fields<S><<<nb, BLOCK, 0, h->stream>>>(h->dp, (const S *)f, (const T *)h->rho, (const T *)h->psi, h->info,
                                                  out);
    });
    LB_HIP_CHECK(hipGetLastError());
}

void launch_sums(lb_handle *h, const void *f) {
    const unsigned nb = dense_blocks(h);
    with_storage(h->prm, [&](auto tag) {
        using S = typename decltype(tag)::type;
        k_sums<S><<<nb, BLOCK, 0, h->stream>>>(h->dp, (const S *)f, h->info, h->partial);
    });
    LB_HIP_CHECK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Batched launches of the fluid stages (see lbm_particles.hip)
// ---------------------------------------------------------------------------
// The sweeps come in a row-aligned and a general instance, launched for the
// members of their kind only (the blocks of the others return at once), so
// neither carries the other's registers.
template <typename S, bool ROWS>
__global__ __launch_bounds__(BLOCK) void kb_density(BatchPlan B) {
    using T = Cmp<S>;
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_DENSE, g)];
    if ((M.rows != 0) != ROWS) return;
    density_body<S, ROWS, false>(M.P, (const S *)M.fin, M.info, (T *)M.rho, (T *)M.psi, M.partial, g, M.D, M.owner,
                                 (const T *)nullptr);
}
// stride: blocks per member, the most fin_blocks() of any member
__global__ __launch_bounds__(FIN_THREADS) void kb_finalize_mass(BatchPlan B, int stride) {
    const int m = (int)(blockIdx.x / stride);
    const BatchMember &M = B.m[m];
    const int *st = B.start + BM_DENSE * (B.nm + 1);
    finalize_body(M.partial, (st[m + 1] - st[m]) * (BLOCK / 64), M.dstate, blockIdx.x % stride);
}
template <typename T>
__global__ __launch_bounds__(SHELL_THREADS) void kb_shell_fill(BatchPlan B) {
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_SPHERE, g)];
    shell_fill_body(M.P, M.D, M.info, (T *)M.rho, (T *)M.psi, (int)g.bid, 0, 1);
}
template <typename S, typename Mo, bool ROWS>
__global__ __launch_bounds__(BLOCK) LBM_COLLIDE_ATTR void kb_collide_stream(BatchPlan B) {
    using T = Cmp<S>;
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_DENSE, g)];
    if ((M.rows != 0) != ROWS) return;
    collide_body<S, Mo, ROWS>(M.P, (const S *)M.fin, (S *)M.fout, (const T *)M.psi, M.info, (T *)M.fsc, g);
}

// density, mass total, virtual fluid and collide sweep of every member
void launch_batch_fluid(const BatchLaunch &L, int parity, hipStream_t s) {
    const BatchPlan &B = L.plan[parity];
    const unsigned nd = (unsigned)L.total[BM_DENSE];
    with_storage(L.prm, [&](auto tag) {
        using S = typename decltype(tag)::type;
        using T = Cmp<S>;
        if (L.any_rows) kb_density<S, true><<<nd, BLOCK, 0, s>>>(B);
        if (L.any_flat) kb_density<S, false><<<nd, BLOCK, 0, s>>>(B);
        kb_finalize_mass<<<(unsigned)(L.nm * L.fin_stride), FIN_THREADS, 0, s>>>(B, L.fin_stride);
        if (L.total[BM_SPHERE] > 0) kb_shell_fill<T><<<(unsigned)L.total[BM_SPHERE], SHELL_THREADS, 0, s>>>(B);
        with_model(L.prm, [&](auto m) {
            if (L.any_rows) kb_collide_stream<S, decltype(m), true><<<nd, BLOCK, 0, s>>>(B);
            if (L.any_flat) kb_collide_stream<S, decltype(m), false><<<nd, BLOCK, 0, s>>>(B);
        });
    });
    LB_HIP_CHECK(hipGetLastError());
}

}  // namespace lbm
