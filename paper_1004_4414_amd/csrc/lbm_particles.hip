// Particle kernels for gfx950 (Secs. III, IV of Jansen & Harting): the
// momentum exchanged on bounce-back links and the Shan-Chen force on the
// virtual fluid summed per sphere, Hertz and lubrication pair forces, the
// leap-frog integration, and the update of the solid map with the covering
// and refilling of sites.
//
// Every per-sphere sum is a fixed-order FP64 block reduction and every list
// is compacted in scan order with wavefront ballots, so results are bitwise
// reproducible.  One block handles one sphere; the only atomics are integer
// (the lowest-index owner of a site, event counters).
#include "lbm_handle.h"

#pragma clang fp contract(off)

namespace lbm {


__device__ __forceinline__ void load3(const double *a, int p, double v[3]) {
    v[0] = a[3 * p];
    v[1] = a[3 * p + 1];
    v[2] = a[3 * p + 2];
}

__device__ __forceinline__ void box_site(int k, const int lo[3], const int ext[3], const DevParams &P, int &x, int &y,
                                         int &z) {
    const int dx = k % ext[0];
    const int t = k / ext[0];
    const int dy = t % ext[1];
    const int dz = t / ext[1];
    x = wrapany(lo[0] + dx, P.nx);
    y = wrapany(lo[1] + dy, P.ny);
    z = wrapany(lo[2] + dz, P.nz);
}

// The sites of a box lo[a] .. lo[a] + ext[a] - 1, numbered k = dx + ext0 (dy
// + ext1 dz), without integer division: the quotients come from FP32
// reciprocals with one correction step (exact below 2^24 sites) and the
// periodic wrap is a conditional add, valid when the box lies within one
// period on either side of [0, L).  Other boxes (tiny lattices) fall back to
// box_site.  `fast` is uniform over the block.
struct BoxWalk {
    int lo[3], ext[3], L[3];
    int e01;
    float r0, r01;
    bool fast;
    __device__ __forceinline__ BoxWalk(const DevParams &P, const int lo_[3], const int ext_[3]) {
        L[0] = P.nx;
        L[1] = P.ny;
        L[2] = P.nz;
        fast = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = lo_[a];
            ext[a] = ext_[a];
            fast = fast && lo[a] >= -L[a] && lo[a] + ext[a] <= 2 * L[a];
        }
        e01 = ext[0] * ext[1];
        fast = fast && (long long)e01 * ext[2] < (1 << 24);
        r0 = ext[0] > 0 ? 1.0f / (float)ext[0] : 0.0f;
        r01 = e01 > 0 ? 1.0f / (float)e01 : 0.0f;
    }
    __device__ __forceinline__ int size() const { return e01 * ext[2]; }
    static __device__ __forceinline__ int qdiv(int k, int d, float r, int &rem) {
        int q = (int)((float)k * r);
        int m = k - q * d;
        if (m < 0) {
            --q;
            m += d;
        } else if (m >= d) {
            ++q;
            m -= d;
        }
        rem = m;
        return q;
    }
    // unwrapped coordinates u and wrapped site coordinates of site k
    __device__ __forceinline__ void site(int k, const DevParams &P, int u[3], int &x, int &y, int &z) const {
        if (!fast) {
            const int dx = k % ext[0], t = k / ext[0];
            u[0] = lo[0] + dx;
            u[1] = lo[1] + t % ext[1];
            u[2] = lo[2] + t / ext[1];
            x = wrapany(u[0], L[0]);
            y = wrapany(u[1], L[1]);
            z = wrapany(u[2], L[2]);
            return;
        }
        int rem, dx;
        const int dz = qdiv(k, e01, r01, rem);
        const int dy = qdiv(rem, ext[0], r0, dx);
        u[0] = lo[0] + dx;
        u[1] = lo[1] + dy;
        u[2] = lo[2] + dz;
        x = wrapc(u[0], L[0]);
        y = wrapc(u[1], L[1]);
        z = wrapc(u[2], L[2]);
    }
};

// box holding the sphere at its previous and its new position (the new one
// unwrapped next to the previous), optionally grown by g sites
__device__ __forceinline__ void union_box(const DevParams &P, const DevParticles &D, int p, int g, int lo[3],
                                          int ext[3]) {
    double Rp[3], Rn[3];
    load3(D.Rprev, p, Rp);
    load3(D.R, p, Rn);
    const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
    for (int a = 0; a < 3; ++a) Rn[a] = Rp[a] + minimg(Rn[a] - Rp[a], L[a]);
    int lo0[3], hi0[3], lo1[3], hi1[3];
    sphere_box(Rp, D.rad[p], lo0, hi0);
    sphere_box(Rn, D.rad[p], lo1, hi1);
    const int Lb[3] = {P.nx, P.ny, P.nz};
    const bool empty = hi0[0] < lo0[0] || hi1[0] < lo1[0];
    for (int a = 0; a < 3; ++a) {
        lo[a] = min(lo0[a], lo1[a]) - g;
        ext[a] = empty ? 0 : min(max(hi0[a], hi1[a]) + g - lo[a] + 1, Lb[a] + 2 * g + 8);
    }
}

// coarse cells touched by the box lo..lo+ext-1 grown by one site, per axis
// (cells[a][0..n[a]), consecutive duplicates removed; a box wider than the
// axis repeats cells, which is harmless); computed by thread 0 into LDS.
// A box spanning more than MAX_AXIS_CELLS cells on an axis sets `wide`.
constexpr int MAX_AXIS_CELLS = 64;
struct AxisCells {
    int n[3];
    int wide;
    int lo[3], ext[3];
    int c[3][MAX_AXIS_CELLS];
};
__device__ __forceinline__ void axis_cells(const DevParams &P, const int lo[3], const int ext[3], AxisCells &ac) {
    const int L[3] = {P.nx, P.ny, P.nz};
    ac.wide = 0;
    for (int a = 0; a < 3; ++a) {
        ac.lo[a] = lo[a] - 1;
        ac.ext[a] = ext[a] > 0 ? ext[a] + 2 : 0;
        int k = 0, last = -1;
        int w = ext[a] > 0 ? wrapany(lo[a] - 1, L[a]) : 0;  // the wrapped coordinate, stepped along
        for (int u = lo[a] - 1; ext[a] > 0 && u <= lo[a] + ext[a]; ++u, w = w + 1 == L[a] ? 0 : w + 1) {
            const int cell = w >> CELL_SHIFT;
            if (cell != last) {
                if (k == MAX_AXIS_CELLS) {
                    ac.wide = 1;
                    break;
                }
                ac.c[a][k++] = cell;
            }
            last = cell;
        }
        ac.n[a] = k;
    }
}
__device__ __forceinline__ long long cell_of(const DevParticles &D, int x, int y, int z) {
    return ((long long)(z >> CELL_SHIFT) * D.cgy + (y >> CELL_SHIFT)) * D.cgx + (x >> CELL_SHIFT);
}
// true in every thread when one of the cells is dirty (block-wide)
__device__ __forceinline__ bool any_dirty(const DevParticles &D, const AxisCells &ac) {
    if (ac.wide) return true;
    const int tot = ac.n[0] * ac.n[1] * ac.n[2];
    int hit = 0;
    for (int k = threadIdx.x; k < tot; k += BLOCK) {
        const int ca = ac.c[0][k % ac.n[0]], cb = ac.c[1][(k / ac.n[0]) % ac.n[1]], cc = ac.c[2][k / (ac.n[0] * ac.n[1])];
        hit |= D.dirty[((long long)cc * D.cgy + cb) * D.cgx + ca] != 0;
    }
    return __syncthreads_or(hit) != 0;
}
__device__ __forceinline__ void mark_dirty(const DevParams &P, const DevParticles &D, const AxisCells &ac) {
    if (ac.wide) {  // site by site over the grown box
        const int V = ac.ext[0] * ac.ext[1] * ac.ext[2];
        for (int k = threadIdx.x; k < V; k += BLOCK) {
            int x, y, z;
            box_site(k, ac.lo, ac.ext, P, x, y, z);
            D.dirty[cell_of(D, x, y, z)] = 1;
        }
        return;
    }
    const int tot = ac.n[0] * ac.n[1] * ac.n[2];
    for (int k = threadIdx.x; k < tot; k += BLOCK) {
        const int ca = ac.c[0][k % ac.n[0]], cb = ac.c[1][(k / ac.n[0]) % ac.n[1]], cc = ac.c[2][k / (ac.n[0] * ac.n[1])];
        D.dirty[((long long)cc * D.cgy + cb) * D.cgx + ca] = 1;
    }
}

__device__ __forceinline__ void new_box(const DevParams &P, const DevParticles &D, int p, int lo[3], int ext[3]) {
    double R[3];
    load3(D.R, p, R);
    int hi[3];
    sphere_box(R, D.rad[p], lo, hi);
    const int Lb[3] = {P.nx, P.ny, P.nz};
    for (int a = 0; a < 3; ++a) ext[a] = hi[a] < lo[a] ? 0 : min(hi[a] - lo[a] + 1, Lb[a] + 8);
}

// ---------------------------------------------------------------------------
// fluid force and torque on each sphere: bounce-back links, Eqs. (13)-(17),
// and the Shan-Chen force on its virtual fluid, Eq. (28).
// The links of sphere p are found from its virtual-fluid sites s: a link
// (x, i) has x = s - c_i fluid (bit opp(i) of the class word of s clear).
// The sweep stored f*_i(x) in the own slot (i, x); this kernel bounces it
// back, Eq. (16): slot (opp(i), s), which x reads as direction opp(i) at the
// next step, receives f_opp(i)(x) = f*_i(x) - w^c with w^c = 6 zeta_i
// rho^c(x) (c_i . u_b) (each link is visited once, by the sphere that owns
// s), and the sphere gains the momentum c_i sum_c (2 f*_i - w^c).
// ---------------------------------------------------------------------------
// The virtual-fluid sites are taken in chunks of BLOCK, one per thread; the
// links of a chunk are numbered by a block scan of their counts, each site
// writes its links into an LDS table at its offset, and they are then
// handled LINKS_PER_PASS per thread with all their loads issued together.
constexpr int LINKS_PER_PASS = 4;

template <typename S, typename T = Cmp<S>>
__device__ __forceinline__ void particle_fluid_force_body(DevParams P, DevParticles D, S *__restrict__ fout,
                                                                const T *__restrict__ rho, const T *__restrict__ fsc,
                                                                const uint32_t *__restrict__ info, const Grid &g) {
    __shared__ double lds[6 * (BLOCK / 64)];
    // the chunk's links in their numbering: (chunk index of the site) << 5 | j
    __shared__ uint16_t lk[BLOCK * (Q - 1)];
    __shared__ unsigned sites[BLOCK];
    __shared__ int sx[BLOCK], sy[BLOCK], sz[BLOCK];
    __shared__ int wtot[BLOCK / 64];
    const int p = g.bid, t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double v[6] = {0, 0, 0, 0, 0, 0};
    double R[3], U[3], W[3];
    load3(D.R, p, R);
    load3(D.U, p, U);
    load3(D.W, p, W);
    if (t < 3) {  // the state of the bounce, for bounced populations formed later
        D.Rl[3 * p + t] = R[t];
        D.Ul[3 * p + t] = U[t];
        D.Wl[3 * p + t] = W[t];
    }
    const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
    const int ns = min(D.shell_cnt[p], D.shell_cap[p]), soff = D.shell_off[p];
    for (int c0 = 0; c0 < ns; c0 += BLOCK) {
        // ---- one virtual-fluid site per thread: Shan-Chen force, link mask
        const int k = c0 + t;
        uint32_t fl = 0;
        unsigned s = 0;
        int x = 0, y = 0, z = 0;
        if (k < ns) {
            s = (unsigned)D.shell[soff + k];
            const uint32_t inf = info[s];
            double F[3];
            if (shell_force_in_slots<S>(inf)) {  // (Fx, Fy) in slot 0, (Fz, 0) in slot j0 of the sweep's output
                const Pair<T> v0 = load_pop(fout, pidx(0, 0, s));
                const Pair<T> v1 = load_pop(fout, pidx(0, shell_force_slot(inf), s));
                F[0] = (double)v0.x;
                F[1] = (double)v0.y;
                F[2] = (double)v1.x;
            } else {
                for (int a = 0; a < 3; ++a) F[a] = (double)fsc[vidx(a, s)];
            }
            site_xyz(s, P, x, y, z);
            const double r[3] = {minimg(x - R[0], L[0]), minimg(y - R[1], L[1]), minimg(z - R[2], L[2])};
            v[0] += F[0];
            v[1] += F[1];
            v[2] += F[2];
            v[3] += r[1] * F[2] - r[2] * F[1];
            v[4] += r[2] * F[0] - r[0] * F[2];
            v[5] += r[0] * F[1] - r[1] * F[0];
            fl = ~inf & 0x7fffeu;  // s + c_j fluid: a link (s + c_j, opp(j))
        }
        // ---- exclusive scan of the link counts (wave shuffles, then waves)
        const int cnt = __popc(fl);
        int inc = cnt;
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(inc, o, 64);
            if (lane >= o) inc += u;
        }
        if (lane == 63) wtot[wave] = inc;
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < BLOCK / 64; ++w) {
            if (w < wave) before += wtot[w];
            total += wtot[w];
        }
        // link numbers before + inc - cnt ... are this site's links, its fluid
        // neighbours j in increasing order
        for (int pos = before + inc - cnt; fl; fl &= fl - 1) lk[pos++] = (uint16_t)((t << 5) | (__ffs(fl) - 1));
        sites[t] = s;
        sx[t] = x;
        sy[t] = y;
        sz[t] = z;
        __syncthreads();
        // ---- the chunk's links, LINKS_PER_PASS per thread per pass
        for (int l0 = t; l0 < total; l0 += LINKS_PER_PASS * BLOCK) {
            unsigned sl[LINKS_PER_PASS], ml[LINKS_PER_PASS];
            int jl[LINKS_PER_PASS], cl[LINKS_PER_PASS];
            bool ok[LINKS_PER_PASS];
            T r0[LINKS_PER_PASS], r1[LINKS_PER_PASS], raw0[LINKS_PER_PASS], raw1[LINKS_PER_PASS];
#pragma unroll
            for (int u = 0; u < LINKS_PER_PASS; ++u) {
                const int l = l0 + u * BLOCK;
                ok[u] = l < total;
                sl[u] = 0;
                ml[u] = 0;
                jl[u] = 1;
                cl[u] = 0;
                if (ok[u]) {
                    const unsigned e = lk[l];
                    const int c = (int)(e >> 5), j = (int)(e & 31u);
                    const int xs = sx[c], ys = sy[c], zs = sz[c];
                    sl[u] = sites[c];
                    jl[u] = j;
                    cl[u] = c;
                    ml[u] = (unsigned)site_of(wrapc(xs + cx(j), P.nx), wrapc(ys + cy(j), P.ny), wrapc(zs + cz(j), P.nz), P);
                }
            }
#pragma unroll
            for (int u = 0; u < LINKS_PER_PASS; ++u) {
                const Pair<T> rr = load_pair(rho, sidx(0, ml[u]));
                const Pair<T> ff = load_pop(fout, pidx(0, opp(jl[u]), ml[u]));  // f*_i(x) in slot (i, x)
                r0[u] = rr.x;
                r1[u] = rr.y;
                raw0[u] = ff.x;
                raw1[u] = ff.y;
            }
#pragma unroll
            for (int u = 0; u < LINKS_PER_PASS; ++u) {
                if (!ok[u]) continue;
                // link (x, i) with x = s + c_j fluid, i = opp(j): f*_i(x), read from slot (i, x), bounces
                // into slot (j, s), where x reads direction j at the next step
                const int j = jl[u], i = opp(j);
                const unsigned ss = sl[u];
                const int x = sx[cl[u]], y = sy[cl[u]], z = sz[cl[u]];
                // lever arm at the link midpoint s - c_i/2 = s + c_j/2
                const double rb[3] = {minimg(x + 0.5 * cx(j) - R[0], L[0]), minimg(y + 0.5 * cy(j) - R[1], L[1]),
                                      minimg(z + 0.5 * cz(j) - R[2], L[2])};
                const double cub = rigid_cu(P, R, U, W, wrapc(x + cx(j), P.nx), wrapc(y + cy(j), P.ny),
                                            wrapc(z + cz(j), P.nz), i);
                T b0, b1, w0, w1;
                bounce_pair<T>(P, cub, i, raw0[u], raw1[u], r0[u], r1[u], b0, b1, w0, w1);
                // the bounced pair goes where x reads direction j at the next
                // step, unless that sweep forms it itself
                if (P.link_write) store_pop_keep(fout, pidx(0, j, ss), b0, b1);
                const double sum = (2.0 * ((double)raw0[u] + zeta(i) * P.rho_ref[0]) - (double)w0) +
                                   (2.0 * ((double)raw1[u] + zeta(i) * P.rho_ref[1]) - (double)w1);
                const double dp[3] = {cx(i) * sum, cy(i) * sum, cz(i) * sum};
                v[0] += dp[0];
                v[1] += dp[1];
                v[2] += dp[2];
                v[3] += rb[1] * dp[2] - rb[2] * dp[1];
                v[4] += rb[2] * dp[0] - rb[0] * dp[2];
                v[5] += rb[0] * dp[1] - rb[1] * dp[0];
            }
        }
        __syncthreads();  // the next chunk rewrites pre, fmask, sites and wtot
    }
    block_sum<6>(v, lds);
    if (t == 0)
        for (int a = 0; a < 3; ++a) {
            D.Ffl[3 * p + a] = v[a];
            D.Tfl[3 * p + a] = v[3 + a];
        }
}

template <typename S, typename T = Cmp<S>>
__global__ __launch_bounds__(BLOCK) void k_particle_fluid_force(DevParams P, DevParticles D, S *__restrict__ fout,
                                                                const T *__restrict__ rho, const T *__restrict__ fsc,
                                                                const uint32_t *__restrict__ info) {
    particle_fluid_force_body<S>(P, D, fout, rho, fsc, info, own_grid());
}

// ---------------------------------------------------------------------------
// pair forces, Eqs. (21) and (22), then the total force and torque: Hertz
// repulsion (5/2) K (r_a + r_b - d)^(3/2) along the centre line, and the
// lubrication contacts (gaps h < h_c) of each sphere, listed in index order.
// The lubrication of Eq. (22), c = 6 pi nu rho0 (r_a r_b/(r_a+r_b))^2 (1/h -
// 1/h_c) with h clamped at h_min, acting on the approach speed, comes in two
// modes (lub_mode):
//  0: the explicit force of Eq. (22) with the latest velocities U(t-1/2),
//     summed here with the Hertz force (the leap-frog then takes it like any
//     other force); unstable where c (1/m_p + 1/m_q) > 2;
//  1: pair impulses in k_integrate: with v* the velocities after every other
//     force, w = n.(v*_p - v*_q) and k_p the number of contacts of sphere p,
//     the pair exchanges J = c w / (1 + c (k_p/m_p + k_q/m_q)) along n (the
//     backward-Euler solution for an isolated pair; sharing a sphere's mass
//     among its contacts keeps simultaneous impulses from overshooting).
// Either way the pair's geometry and c are computed from the lower index to
// the higher, so both ends use identical values.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pair_forces_body(DevParams P, DevParticles D, DevState *st, const Grid &g) {
    __shared__ double lds[3 * (BLOCK / 64)];
    __shared__ int clds[8];
    const int p = g.bid;
    double Rp[3];
    load3(D.R, p, Rp);
    const double rp = D.rad[p];
    const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
    double F[3] = {0, 0, 0};
    int ncont = 0;
    int nnb = 0;  // neighbours for the map update (index order)
    double nu = 0.0;  // mean kinematic viscosity of the two components
    for (int c = 0; c < 2; ++c) nu += (1.0 / 3.0) * (P.tau[c] - 0.5);
    nu /= 2.0;
    for (int q0 = 0; q0 < P.np; q0 += BLOCK) {
        const int q = q0 + threadIdx.x;
        bool lub = false, nb = false;
        if (q < P.np && q != p) {
            double d[3], dist2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                d[a] = minimg(D.R[3 * q + a] - Rp[a], L[a]);
                dist2 += d[a] * d[a];
            }
            const double rsum = rp + D.rad[q];
            nb = dist2 < (rsum + NB_REACH) * (rsum + NB_REACH);
            const double reach = rsum + (P.lub_hc > 0.0 ? P.lub_hc : 0.0);
            if (dist2 < reach * reach) {
                const double dist = sqrt(dist2);
                if (dist > 0.0) {
                    if (dist < rsum) {
                        const double fh = 2.5 * P.k_hertz * pow(rsum - dist, 1.5);
                        for (int a = 0; a < 3; ++a) F[a] -= fh * d[a] / dist;
                    }
                    lub = P.lub_hc > 0.0 && dist - rsum < P.lub_hc;
                }
            }
        }
        const int nslot = block_compact(nb, nnb, clds);
        if (nb && nslot < NB_CAP) D.nbr[(size_t)p * NB_CAP + nslot] = q;
        const int slot = block_compact(lub, ncont, clds);
        if (lub && (P.lub_mode == 0 || slot < MAX_LUB_CONTACTS)) {
            // the pair's geometry as both ends compute it: from the lower index to the higher
            const int lo = min(p, q), hi = max(p, q);
            double d[3], dist2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                d[a] = minimg(D.R[3 * hi + a] - D.R[3 * lo + a], L[a]);
                dist2 += d[a] * d[a];
            }
            const double dist = sqrt(dist2);
            const double rsum = D.rad[lo] + D.rad[hi];
            const double h = dist - rsum;
            const double hh = h < P.lub_hmin ? P.lub_hmin : h;
            const double ared = D.rad[lo] * D.rad[hi] / rsum;
            const double c = 6.0 * M_PI * nu * P.rho0 * ared * ared * (1.0 / hh - 1.0 / P.lub_hc);
            if (P.lub_mode == 0) {
                // explicit force, Eq. (22): -c n [n.(U_lo - U_hi)] on lo, the opposite on hi
                double w = 0.0;
                for (int a = 0; a < 3; ++a) w += d[a] / dist * (D.U[3 * lo + a] - D.U[3 * hi + a]);
                const double sgn = p == lo ? -1.0 : 1.0;
                for (int a = 0; a < 3; ++a) F[a] += sgn * (c * w) * (d[a] / dist);
            } else {
                const size_t e = (size_t)p * MAX_LUB_CONTACTS + slot;
                D.cont[e] = q;
                D.cont_c[e] = c;
                for (int a = 0; a < 3; ++a) D.cont_n[3 * e + a] = d[a] / dist;
            }
        }
    }
    block_sum<3>(F, lds);
    if (threadIdx.x == 0) {
        D.nnbr[p] = nnb;
        D.ncont[p] = P.lub_mode == 0 ? 0 : min(ncont, MAX_LUB_CONTACTS);
        if (P.lub_mode != 0 && ncont > MAX_LUB_CONTACTS) atomicOr(&st->overflow, 16);
        for (int a = 0; a < 3; ++a) {
            D.Ftot[3 * p + a] = F[a];  // the pair forces; k_forces_total adds the rest
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_pair_forces(DevParams P, DevParticles D, DevState *st) {
    pair_forces_body(P, D, st, own_grid());
}

// ---------------------------------------------------------------------------
// The same pair forces from a cell list (cells at least 2 r_max + h_c wide, at
// least 3 per axis, so every partner within reach lies in the 27 cells around
// a sphere and no cell is visited twice).  The list is a counting sort with
// integer atomics; the candidates of a sphere are sorted by index before use,
// so contacts are listed in index order and the force sums run in a fixed
// order whatever the order inside a cell.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pair_cell(const DevParams &P, const DevParticles &D, int p) {
    const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
    const int g[3] = {D.pgx, D.pgy, D.pgz};
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double r = D.R[3 * p + a];
        int k = isfinite(r) ? (int)(r / L[a] * g[a]) : 0;
        c[a] = k < 0 ? 0 : (k >= g[a] ? g[a] - 1 : k);
    }
    return (c[2] * g[1] + c[1]) * g[0] + c[0];
}

__device__ __forceinline__ void pcell_count_body(DevParams P, DevParticles D, const Grid &g) {
    const int p = g.bid * BLOCK + threadIdx.x;
    if (p >= P.np) return;
    const int c = pair_cell(P, D, p);
    D.pc_of[p] = c;
    atomicAdd(&D.pc_cnt[c], 1);
}

__global__ void k_pcell_count(DevParams P, DevParticles D) {
    pcell_count_body(P, D, own_grid());
}

// exclusive scan of the cell counts (one block: contiguous runs per thread,
// then a scan of the run totals)
constexpr int PCS_THREADS = 1024;
__device__ __forceinline__ void pcell_scan_body(DevParticles D, const Grid &g) {
    __shared__ int tot[PCS_THREADS];
    const int nc = D.pgx * D.pgy * D.pgz;
    const int t = threadIdx.x;
    const int run = (nc + PCS_THREADS - 1) / PCS_THREADS;
    const int a = min(nc, t * run), b = min(nc, a + run);
    int sum = 0;
    for (int k = a; k < b; ++k) sum += D.pc_cnt[k];
    tot[t] = sum;
    __syncthreads();
    for (int o = 1; o < PCS_THREADS; o <<= 1) {
        const int v = t >= o ? tot[t - o] : 0;
        __syncthreads();
        tot[t] += v;
        __syncthreads();
    }
    int base = tot[t] - sum;
    for (int k = a; k < b; ++k) {
        D.pc_start[k] = base;
        base += D.pc_cnt[k];
    }
    if (t == PCS_THREADS - 1) D.pc_start[nc] = tot[t];
}

__global__ __launch_bounds__(PCS_THREADS) void k_pcell_scan(DevParticles D) {
    pcell_scan_body(D, own_grid());
}

// scatter into the cells; counting down leaves the counts at zero for the next step
__device__ __forceinline__ void pcell_fill_body(DevParams P, DevParticles D, const Grid &g) {
    const int p = g.bid * BLOCK + threadIdx.x;
    if (p >= P.np) return;
    const int c = D.pc_of[p];
    const int k = atomicSub(&D.pc_cnt[c], 1) - 1;
    D.pc_items[D.pc_start[c] + k] = p;
}

__global__ void k_pcell_fill(DevParams P, DevParticles D) {
    pcell_fill_body(P, D, own_grid());
}

constexpr int PAIR_MAX_CAND = 512;  // partners within the 27 cells of one sphere
__device__ __forceinline__ void pair_forces_cells_body(DevParams P, DevParticles D, DevState *st, const Grid &g) {
    __shared__ int cand[PAIR_MAX_CAND];
    __shared__ int cstart[27], ccount[27], coff[28];
    const int p = g.bid, t = threadIdx.x;
    double Rp[3];
    load3(D.R, p, Rp);
    const double rp = D.rad[p];
    const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
    double nu = 0.0;  // mean kinematic viscosity of the two components
    for (int c = 0; c < 2; ++c) nu += (1.0 / 3.0) * (P.tau[c] - 0.5);
    nu /= 2.0;
    // the 27 cells around the sphere's cell and their runs
    const int c0 = D.pc_of[p];
    const int gx = D.pgx, gy = D.pgy, gz = D.pgz;
    if (t < 27) {
        const int cx0 = c0 % gx, cy0 = (c0 / gx) % gy, cz0 = c0 / (gx * gy);
        const int ux = wrapc(cx0 + t % 3 - 1, gx), uy = wrapc(cy0 + (t / 3) % 3 - 1, gy), uz = wrapc(cz0 + t / 9 - 1, gz);
        const int c = (uz * gy + uy) * gx + ux;
        cstart[t] = D.pc_start[c];
        ccount[t] = D.pc_start[c + 1] - D.pc_start[c];
    }
    __syncthreads();
    if (t == 0) {
        coff[0] = 0;
        for (int k = 0; k < 27; ++k) coff[k + 1] = coff[k] + ccount[k];
    }
    __syncthreads();
    const int K = coff[27];
    if (K > PAIR_MAX_CAND) {
        if (t == 0) {
            D.ncont[p] = 0;
            D.nnbr[p] = NB_CAP + 1;  // unknown: the map update tests every sphere
            for (int a = 0; a < 3; ++a) D.Ftot[3 * p + a] = 0.0;
            atomicOr(&st->overflow, 16);
        }
        return;
    }
    for (int k = 0; k < 27; ++k)
        for (int j = t; j < ccount[k]; j += 64) cand[coff[k] + j] = D.pc_items[cstart[k] + j];
    // pad to a power of two and sort ascending (bitonic)
    int n2 = 1;
    while (n2 < K) n2 <<= 1;
    for (int j = K + t; j < n2; j += 64) cand[j] = 0x7fffffff;
    __syncthreads();
    for (int size = 2; size <= n2; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int j = t; j < n2; j += 64) {
                const int partner = j ^ stride;
                if (partner > j) {
                    const bool up = (j & size) == 0;
                    const int a = cand[j], b = cand[partner];
                    if ((a > b) == up) {
                        cand[j] = b;
                        cand[partner] = a;
                    }
                }
            }
            __syncthreads();
        }
    double F[3] = {0, 0, 0};
    int ncont = 0;
    int nnb = 0;  // neighbours for the map update (index order: the candidates are sorted)
    for (int j0 = 0; j0 < K; j0 += 64) {
        const int j = j0 + t;
        const int q = j < K ? cand[j] : -1;
        bool lub = false, nb = false;
        if (q >= 0 && q != p) {
            double d[3], dist2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                d[a] = minimg(D.R[3 * q + a] - Rp[a], L[a]);
                dist2 += d[a] * d[a];
            }
            const double rsum = rp + D.rad[q];
            nb = dist2 < (rsum + NB_REACH) * (rsum + NB_REACH);
            const double reach = rsum + (P.lub_hc > 0.0 ? P.lub_hc : 0.0);
            if (dist2 < reach * reach) {
                const double dist = sqrt(dist2);
                if (dist > 0.0) {
                    if (dist < rsum) {
                        const double fh = 2.5 * P.k_hertz * pow(rsum - dist, 1.5);
                        for (int a = 0; a < 3; ++a) F[a] -= fh * d[a] / dist;
                    }
                    lub = P.lub_hc > 0.0 && dist - rsum < P.lub_hc;
                }
            }
        }
        const unsigned long long below = (t == 0) ? 0ull : (~0ull >> (64 - t));
        const unsigned long long nball = __ballot(nb);
        const int nslot = nnb + __popcll(nball & below);
        nnb += __popcll(nball);
        if (nb && nslot < NB_CAP) D.nbr[(size_t)p * NB_CAP + nslot] = q;
        const unsigned long long ball = __ballot(lub);
        const int slot = ncont + __popcll(ball & below);
        ncont += __popcll(ball);
        if (lub && (P.lub_mode == 0 || slot < MAX_LUB_CONTACTS)) {
            // the pair's geometry as both ends compute it: from the lower index to the higher
            const int lo = min(p, q), hi = max(p, q);
            double d[3], dist2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                d[a] = minimg(D.R[3 * hi + a] - D.R[3 * lo + a], L[a]);
                dist2 += d[a] * d[a];
            }
            const double dist = sqrt(dist2);
            const double rsum = D.rad[lo] + D.rad[hi];
            const double h = dist - rsum;
            const double hh = h < P.lub_hmin ? P.lub_hmin : h;
            const double ared = D.rad[lo] * D.rad[hi] / rsum;
            const double c = 6.0 * M_PI * nu * P.rho0 * ared * ared * (1.0 / hh - 1.0 / P.lub_hc);
            if (P.lub_mode == 0) {
                // explicit force, Eq. (22): -c n [n.(U_lo - U_hi)] on lo, the opposite on hi
                double w = 0.0;
                for (int a = 0; a < 3; ++a) w += d[a] / dist * (D.U[3 * lo + a] - D.U[3 * hi + a]);
                const double sgn = p == lo ? -1.0 : 1.0;
                for (int a = 0; a < 3; ++a) F[a] += sgn * (c * w) * (d[a] / dist);
            } else {
                const size_t e = (size_t)p * MAX_LUB_CONTACTS + slot;
                D.cont[e] = q;
                D.cont_c[e] = c;
                for (int a = 0; a < 3; ++a) D.cont_n[3 * e + a] = d[a] / dist;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
        for (int off = 32; off > 0; off >>= 1) F[a] += __shfl_down(F[a], off, 64);
    if (t == 0) {
        D.nnbr[p] = nnb;
        D.ncont[p] = P.lub_mode == 0 ? 0 : min(ncont, MAX_LUB_CONTACTS);
        if (P.lub_mode != 0 && ncont > MAX_LUB_CONTACTS) atomicOr(&st->overflow, 16);
        for (int a = 0; a < 3; ++a) {
            D.Ftot[3 * p + a] = F[a];  // the pair forces; k_forces_total adds the rest
        }
    }
}

__global__ __launch_bounds__(64) void k_pair_forces_cells(DevParams P, DevParticles D, DevState *st) {
    pair_forces_cells_body(P, D, st, own_grid());
}

// total force and torque of each sphere (fluid, pending impulses, pair forces
// in that order of summation) and its velocity after every force but the
// lubrication impulses.  With force_avg the fluid part is the mean of this
// step's and the previous step's (this step's alone while no previous one is
// kept); the previous one is kept in either case.
__device__ __forceinline__ void forces_total_body(DevParams P, DevParticles D, const Grid &g) {
    const int p = g.bid * BLOCK + threadIdx.x;
    if (p >= P.np) return;
    for (int a = 0; a < 3; ++a) {
        double ff = D.Ffl[3 * p + a], tf = D.Tfl[3 * p + a];
        const double fp = D.Fprev[6 * p + a], tp = D.Fprev[6 * p + 3 + a];
        D.Fprev[6 * p + a] = ff;
        D.Fprev[6 * p + 3 + a] = tf;
        if (P.force_avg && !isnan(fp)) {
            ff = 0.5 * (ff + fp);
            tf = 0.5 * (tf + tp);
        }
        D.Ftot[3 * p + a] = ff + D.P[3 * p + a] + D.Ftot[3 * p + a];
        D.Ttot[3 * p + a] = tf + D.PT[3 * p + a];
        D.vs[3 * p + a] = D.U[3 * p + a] + (D.prescribed[p] ? 0.0 : D.Ftot[3 * p + a] / D.mass[p]);
    }
}

__global__ void k_forces_total(DevParams P, DevParticles D) {
    forces_total_body(P, D, own_grid());
}

// lubrication impulses, then the leap-frog of Eqs. (9), (10):
// U(t+1/2) = v* + impulses / m, R(t+1) = R(t) + U, Omega(t+1/2) = Omega(t-1/2)
// + D/J; the pending impulses are consumed
__device__ __forceinline__ void integrate_body(DevParams P, DevParticles D, DevState *st, const Grid &g) {
    const int p = g.bid * BLOCK + threadIdx.x;
    if (p >= P.np) return;
    const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
    double imp[3] = {0, 0, 0};
    const int kp = D.ncont[p];
    const double inv_p = D.prescribed[p] ? 0.0 : kp / D.mass[p];
    for (int k = 0; k < kp; ++k) {
        const size_t e = (size_t)p * MAX_LUB_CONTACTS + k;
        const int q = D.cont[e];
        const int lo = min(p, q), hi = max(p, q);
        const double c = D.cont_c[e];
        const double n[3] = {D.cont_n[3 * e], D.cont_n[3 * e + 1], D.cont_n[3 * e + 2]};
        double w = 0.0;
        for (int a = 0; a < 3; ++a) w += n[a] * (D.vs[3 * lo + a] - D.vs[3 * hi + a]);
        const double inv_q = D.prescribed[q] ? 0.0 : D.ncont[q] / D.mass[q];
        const double J = c * w / (1.0 + c * (p == lo ? inv_p + inv_q : inv_q + inv_p));
        const double sgn = p == lo ? -1.0 : 1.0;
        for (int a = 0; a < 3; ++a) imp[a] += sgn * J * n[a];
    }
    bool fast = false;
    for (int a = 0; a < 3; ++a) {
        D.Ftot[3 * p + a] += imp[a];
        if (!D.prescribed[p]) {
            D.U[3 * p + a] = D.vs[3 * p + a] + imp[a] / D.mass[p];
            D.W[3 * p + a] += D.Ttot[3 * p + a] / D.inertia[p];
        }
        double r = D.R[3 * p + a] + D.U[3 * p + a];
        if (r >= L[a]) r -= L[a];
        if (r < 0.0) r += L[a];
        D.R[3 * p + a] = r;
        D.P[3 * p + a] = 0.0;
        D.PT[3 * p + a] = 0.0;
        // the map update takes moves below one site per step along each axis
        fast = fast || !(fabs(D.U[3 * p + a]) < 1.0);
    }
    if (fast) atomicOr(&st->overflow, 8);
}

__global__ void k_integrate(DevParams P, DevParticles D, DevState *st) {
    integrate_body(P, D, st, own_grid());
}

// exclusive prefix sum of v over the block (in thread order) and its total;
// lds: at least BLOCK/64 ints
__device__ __forceinline__ int block_scan_excl(int v, int &total, int *lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    int before = 0;
    total = 0;
    for (int w = 0; w < BLOCK / 64; ++w) {
        const int c = lds[w];
        if (w < wave) before += c;
        total += c;
    }
    __syncthreads();
    return before + inc - v;
}

// ---------------------------------------------------------------------------
// Solid map (Sec. III): a site belongs to the lowest-index sphere whose
// centre, rounded to 2^-20, is closer than its rounded radius.
//
// The full classification (new spheres, restored states) marks every site
// inside sphere p with p in stage[] (lowest index wins) and k_map_commit_full
// turns the marks into owners.  The per-step update is incremental: a site can
// change owner only if it changes side of some sphere's surface.  For each
// sphere those sites are found exactly, among its candidate sites while the
// centre stays within the margin of the last scan, else by scanning the box
// of its old and new positions.  Each such site's new owner is the lowest
// index among that sphere and its listed neighbours that contain the site at
// their new positions, so the map always equals a full classification at the
// current positions.
// ---------------------------------------------------------------------------

// the band half-width of the candidate sites: about 192 of them
__device__ __forceinline__ double cand_tau(double r) { return fmin(0.5, 192.0 / (8.0 * M_PI * r * r)); }

// sphere q (current position) contains site (x, y, z)
__device__ __forceinline__ bool sphere_holds(const DevParams &P, const DevParticles &D, int q, int x, int y, int z) {
    long long cq[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) cq[a] = fixed20(D.R[3 * q + a]);
    const long long rq = fixed20(D.rad[q]);
    return dist2_sphere(x, y, z, cq, P.nx, P.ny, P.nz) < rq * rq;
}

// full classification of sphere p: marks and candidate sites
__device__ __forceinline__ void map_mark_body(DevParams P, DevParticles D, int32_t *__restrict__ stage, const Grid &g) {
    const int p = g.bid;
    long long cq[3];
    for (int a = 0; a < 3; ++a) cq[a] = fixed20(D.R[3 * p + a]);
    const long long rq = fixed20(D.rad[p]);
    const long long r2q = rq * rq;
    int lo[3], ext[3];
    new_box(P, D, p, lo, ext);
    const BoxWalk bw(P, lo, ext);
    const bool near = near_box(lo, ext, cq, P);
    const int V = bw.size();
    __shared__ int lds[BLOCK / 64 + 1];
    const double tau = cand_tau(D.rad[p]);
    int32_t *cd = D.cand + (size_t)p * CAND_CAP;
    int nc = 0;
    for (int k0 = 0; k0 < V; k0 += BLOCK) {
        const int k = k0 + threadIdx.x;
        bool near_surface = false;
        long long n = 0;
        if (k < V) {
            int u[3], x, y, z;
            bw.site(k, P, u, x, y, z);
            const long long d2 = near ? dist2_unwrapped(u, cq) : dist2_sphere(x, y, z, cq, P.nx, P.ny, P.nz);
            n = site_of(x, y, z, P);
            if (d2 < r2q) atomicMin(&stage[n], p);
            near_surface = fabs(sqrt((double)d2) - (double)rq) * (1.0 / 1048576.0) < tau;
        }
        const int slot = block_compact(near_surface, nc, lds);
        if (near_surface && slot < CAND_CAP) cd[slot] = (int32_t)n;
    }
    if (threadIdx.x == 0) {
        D.ncand[p] = min(nc, CAND_CAP);
        D.margin[p] = nc <= CAND_CAP ? tau : 0.0;  // a full list only: else every update scans
    }
}

__global__ __launch_bounds__(BLOCK) void k_map_mark(DevParams P, DevParticles D, int32_t *__restrict__ stage) {
    map_mark_body(P, D, stage, own_grid());
}

// The sites of sphere p that change side between the centre of the last map
// update (Rprev) and the new one (R).  A site whose owner changes gets the new
// owner in stage[] and goes into p's change list; a fluid site that p takes is
// one of p's covered sites, a site of p that no sphere takes one of its
// uncovered sites (Eqs. (18)-(20)).  Lists are in scan order.
__device__ __forceinline__ void map_flip_body(DevParams P, DevParticles D, const int32_t *__restrict__ owner,
                                              int32_t *__restrict__ stage, uint32_t *__restrict__ info, DevState *st,
                                              const Grid &g) {
    const int p = g.bid;
    {  // the blocks also clear the coarse dirty cells of the previous step, a slice each
        const int ncell = D.cgx * D.cgy * D.cgz;
        const int per = (ncell + (int)g.nb - 1) / (int)g.nb;
        for (int c = p * per + threadIdx.x; c < min(ncell, (p + 1) * per); c += BLOCK) D.dirty[c] = 0;
    }
    if (D.track_flags) {  // the flags of the words the previous update recomputed
        const int off = 2 * D.ev_off[p], n = min(D.chg_prev_cnt[p], 2 * D.ev_cap[p]);
        for (int k = threadIdx.x; k < n * Q; k += BLOCK) {
            const int e = k / Q, i = k - e * Q;
            int x, y, z;
            site_xyz(D.chg_prev[off + e], P, x, y, z);
            info[site_of(wrapc(x + cx(i), P.nx), wrapc(y + cy(i), P.ny), wrapc(z + cz(i), P.nz), P)] &= ~INFO_FLAG;
        }
    }
    long long cn[3], co[3];
    for (int a = 0; a < 3; ++a) {
        cn[a] = fixed20(D.R[3 * p + a]);
        co[a] = fixed20(D.Rprev[3 * p + a]);
    }
    const long long rq = fixed20(D.rad[p]);
    const long long r2q = rq * rq;
    // The candidates hold every site that can change side while both centres
    // are closer than the margin to the centre of the last scan: a site on
    // different sides for the two is within that distance of that sphere's
    // surface.  The old centre is (it was the last scan, or passed this test).
    bool cand_ok = true;
    {
        long long d2 = 0;
        for (int a = 0; a < 3; ++a) {
            const long long Lq = (long long)(a == 0 ? P.nx : (a == 1 ? P.ny : P.nz)) << 20;
            long long d = cn[a] - fixed20(D.Rscan[3 * p + a]);
            if (d > Lq / 2) d -= Lq;
            else if (d <= -(Lq / 2)) d += Lq;
            d2 += d * d;
            cand_ok = cand_ok && fabs(D.U[3 * p + a]) < 1.0;
        }
        cand_ok = cand_ok && sqrt((double)d2) * (1.0 / 1048576.0) < D.margin[p] - 1e-9;
    }
    __shared__ int lds[BLOCK / 64 + 1];
    const int eoff = D.ev_off[p], ecap = D.ev_cap[p];
    const int coff = 2 * eoff, ccap = 2 * ecap;
    const int nnb = D.nnbr[p];
    const int32_t *nb = D.nbr + (size_t)p * NB_CAP;
    int ncov = 0, nunc = 0, nchg = 0;
    // one site per thread (flip: it changes side of p); every thread calls
    auto settle = [&](bool flip, bool in_new, long long n, int x, int y, int z) {
        if (!__syncthreads_or(flip)) return;  // most chunks have no flip
        bool chg = false, cov = false, unc = false;
        if (flip) {
            int best = in_new ? p : 0x7fffffff;
            if (nnb <= NB_CAP) {
                for (int k = 0; k < nnb; ++k) {
                    const int q = nb[k];
                    if (q < best && sphere_holds(P, D, q, x, y, z)) best = q;
                }
            } else {
                for (int q = 0; q < min(best, P.np); ++q)
                    if (q != p && sphere_holds(P, D, q, x, y, z)) {
                        best = q;
                        break;
                    }
            }
            const int32_t nw = best == 0x7fffffff ? OWN_FLUID : best;
            const int32_t o = owner[n];
            chg = nw != o;
            cov = chg && o == OWN_FLUID && nw == p;
            unc = chg && o == p && nw == OWN_FLUID;
            if (chg) stage[n] = nw == OWN_FLUID ? STAGE_FLUID : nw;  // the same value from every block
        }
        // the three list slots from one block scan of packed 10-bit flags
        int total;
        const int pre = block_scan_excl((int)chg | ((int)cov << 10) | ((int)unc << 20), total, lds);
        if (chg && nchg + (pre & 1023) < ccap) D.chg[coff + nchg + (pre & 1023)] = (int32_t)n;
        if (cov && ncov + ((pre >> 10) & 1023) < ecap) D.cov[eoff + ncov + ((pre >> 10) & 1023)] = (int32_t)n;
        if (unc && nunc + (pre >> 20) < ecap) D.unc[eoff + nunc + (pre >> 20)] = (int32_t)n;
        nchg += total & 1023;
        ncov += (total >> 10) & 1023;
        nunc += total >> 20;
    };
    if (cand_ok) {  // uniform over the block
        const int nc = D.ncand[p];
        const int32_t *cd = D.cand + (size_t)p * CAND_CAP;
        for (int k0 = 0; k0 < nc; k0 += BLOCK) {
            const int k = k0 + threadIdx.x;
            bool flip = false, in_new = false;
            long long n = 0;
            int x = 0, y = 0, z = 0;
            if (k < nc) {
                n = cd[k];
                site_xyz(n, P, x, y, z);
                in_new = dist2_sphere(x, y, z, cn, P.nx, P.ny, P.nz) < r2q;
                flip = in_new != (dist2_sphere(x, y, z, co, P.nx, P.ny, P.nz) < r2q);
            }
            settle(flip, in_new, n, x, y, z);
        }
    } else {
        // scan the box of both positions; new candidates around the new centre
        int lo[3], ext[3];
        union_box(P, D, p, 0, lo, ext);
        const BoxWalk bw(P, lo, ext);
        const int V = bw.size();
        const double tau = cand_tau(D.rad[p]);
        int32_t *cd = D.cand + (size_t)p * CAND_CAP;
        int nc = 0;
        for (int k0 = 0; k0 < V; k0 += BLOCK) {
            const int k = k0 + threadIdx.x;
            bool flip = false, in_new = false, near_surface = false;
            long long n = 0;
            int x = 0, y = 0, z = 0;
            if (k < V) {
                int u[3];
                bw.site(k, P, u, x, y, z);
                n = site_of(x, y, z, P);
                const long long d2 = dist2_sphere(x, y, z, cn, P.nx, P.ny, P.nz);
                in_new = d2 < r2q;
                flip = in_new != (dist2_sphere(x, y, z, co, P.nx, P.ny, P.nz) < r2q);
                near_surface = fabs(sqrt((double)d2) - (double)rq) * (1.0 / 1048576.0) < tau;
            }
            const int slot = block_compact(near_surface, nc, lds);
            if (near_surface && slot < CAND_CAP) cd[slot] = (int32_t)n;
            settle(flip, in_new, n, x, y, z);
        }
        if (threadIdx.x == 0) {
            D.ncand[p] = min(nc, CAND_CAP);
            D.margin[p] = nc <= CAND_CAP ? tau : 0.0;
            for (int a = 0; a < 3; ++a) D.Rscan[3 * p + a] = D.R[3 * p + a];
        }
    }
    __syncthreads();  // every thread has read Rprev
    if (threadIdx.x == 0) {
        for (int a = 0; a < 3; ++a) D.Rprev[3 * p + a] = D.R[3 * p + a];
        D.cov_cnt[p] = ncov;
        D.unc_cnt[p] = nunc;
        D.chg_cnt[p] = nchg;
        if (ncov > ecap || nunc > ecap || nchg > ccap) atomicOr(&st->overflow, 4);
    }
}

__global__ __launch_bounds__(BLOCK) void k_map_flip(DevParams P, DevParticles D, const int32_t *__restrict__ owner,
                                                    int32_t *__restrict__ stage, uint32_t *__restrict__ info,
                                                    DevState *st) {
    map_flip_body(P, D, owner, stage, info, st, own_grid());
}

// The bounced pairs of every sphere link of fluid site n (class word inf),
// written into the solid sites' slots of f as the link kernel writes them:
// from f*_i(n) in slot (i, n), the density deviations of n in rho, and the
// sphere state of the bounce.
template <typename S>
__device__ __forceinline__ void write_site_bounces(const DevParams &P, const DevParticles &D, S *__restrict__ f,
                                                   const Cmp<S> *__restrict__ rho, const int32_t *__restrict__ owner,
                                                   long long n, int x, int y, int z, uint32_t inf) {
    using T = Cmp<S>;
    const Pair<T> dr = load_pair(rho, sidx(0, (unsigned)n));
    uint32_t bits = inf & 0x7fffeu;
    while (bits) {
        const int i = __ffs(bits) - 1;
        bits &= bits - 1;
        const long long s = site_of(wrapc(x + cx(i), P.nx), wrapc(y + cy(i), P.ny), wrapc(z + cz(i), P.nz), P);
        const int32_t q = owner[s];
        if (q < 0) continue;  // walls: the wall kernel writes their links
        double R[3], U[3], W[3];
        load3(D.Rl, q, R);
        load3(D.Ul, q, U);
        load3(D.Wl, q, W);
        const Pair<T> raw = load_pop(f, pidx(0, i, (unsigned)n));
        T b0, b1, w0, w1;
        bounce_pair<T>(P, rigid_cu(P, R, U, W, x, y, z, i), i, raw.x, raw.y, dr.x, dr.y, b0, b1, w0, w1);
        store_pop_keep(f, pidx(0, opp(i), (unsigned)s), b0, b1);
    }
}

// When the next sweep forms the bounced populations itself, the links of
// the fluid sites that a map change touches (a changed site and its 18
// neighbours, fluid on the map of the bounce) are written out here instead,
// before covering and refilling read or overwrite their slots; the next
// sweep finds these sites flagged in their class words and pulls plainly.
template <typename S>
__device__ __forceinline__ void map_fixup_body(DevParams P, DevParticles D, S *__restrict__ f,
                                               const Cmp<S> *__restrict__ rho, const int32_t *__restrict__ owner,
                                               const uint32_t *__restrict__ info, const Grid &g) {
    const int p = g.bid;
    const int off = 2 * D.ev_off[p], n = min(D.chg_cnt[p], 2 * D.ev_cap[p]);
    for (int k = threadIdx.x; k < n * Q; k += BLOCK) {
        const int e = k / Q, i = k - e * Q;
        int x, y, z;
        site_xyz(D.chg[off + e], P, x, y, z);
        x = wrapc(x + cx(i), P.nx);
        y = wrapc(y + cy(i), P.ny);
        z = wrapc(z + cz(i), P.nz);
        const long long m = site_of(x, y, z, P);
        if (owner[m] != OWN_FLUID) continue;
        const uint32_t inf = info[m];
        if (inf & 0x7fffeu) write_site_bounces<S>(P, D, f, rho, owner, m, x, y, z, inf);
    }
}

template <typename S>
__global__ __launch_bounds__(BLOCK) void k_map_fixup(DevParams P, DevParticles D, S *__restrict__ f,
                                                     const Cmp<S> *__restrict__ rho,
                                                     const int32_t *__restrict__ owner,
                                                     const uint32_t *__restrict__ info) {
    map_fixup_body<S>(P, D, f, rho, owner, info, own_grid());
}

// Every pending bounced population written out (before a plain reader of
// the populations: observables, fields, state, a batch): the fluid sites
// with links whose class word is not flagged (the flagged ones were written
// by the fix-up).
template <typename S>
__global__ __launch_bounds__(BLOCK) void k_materialize(DevParams P, DevParticles D, S *__restrict__ f,
                                                       const Cmp<S> *__restrict__ rho,
                                                       const int32_t *__restrict__ owner,
                                                       const uint32_t *__restrict__ info) {
    const long long n = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= P.N) return;
    const uint32_t inf = info[n];
    if (site_class(inf) != CLS_FLUID || (inf & INFO_FLAG) || !(inf & 0x7fffeu)) return;
    int x, y, z;
    site_xyz(n, P, x, y, z);
    write_site_bounces<S>(P, D, f, rho, owner, n, x, y, z, inf);
}

// Covering, Eq. (18): the fluid of a covered site is removed and its momentum
// goes to the sphere.  Refilling, Eqs. (23)-(26), (31): an uncovered site gets
// f^eq(rho_new, u_surf) with rho_new^c the mean of rho^c(t+1) over its
// neighbours that are fluid before and after the move, scaled by the mass
// correction; the sphere loses the created momentum.  Both impulses are
// applied in the next step's integration.
template <typename S>
__device__ __forceinline__ void cover_refill_body(DevParams P, DevParticles D, S *__restrict__ f,
                                                        const int32_t *__restrict__ owner,
                                                        const int32_t *__restrict__ stage, DevState *st, const Grid &g) {
    __shared__ double lds[6 * (BLOCK / 64)];
    const int p = g.bid;
    const long long N = P.N;
    const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
    double R[3], U[3], W[3];
    load3(D.R, p, R);
    load3(D.U, p, U);
    load3(D.W, p, W);
    double v[6] = {0, 0, 0, 0, 0, 0};
    const int off = D.ev_off[p], cap = D.ev_cap[p];
    const int nc = min(D.cov_cnt[p], cap), nu = min(D.unc_cnt[p], cap);
    if (nc == 0 && nu == 0) return;  // uniform over the block
    for (int k = threadIdx.x; k < nc; k += BLOCK) {
        const long long n = D.cov[off + k];
        int x, y, z;
        site_xyz(n, P, x, y, z);
        // f_i(y) = slot (i, y - c_i); the reference part of the stored values
        // has no momentum.  Nothing reads those slots once y is solid.
        double mom[3] = {0, 0, 0};
        for (int i = 0; i < Q; ++i) {
            const long long src = site_of(wrapc(x - cx(i), P.nx), wrapc(y - cy(i), P.ny), wrapc(z - cz(i), P.nz), P);
            const auto d2 = load_pop(f, pidx(0, i, (unsigned)src));
            const double di = (double)d2.x + (double)d2.y;
            mom[0] += di * cx(i);
            mom[1] += di * cy(i);
            mom[2] += di * cz(i);
        }
        const double r[3] = {minimg(x - R[0], L[0]), minimg(y - R[1], L[1]), minimg(z - R[2], L[2])};
        for (int a = 0; a < 3; ++a) v[a] += mom[a];
        v[3] += r[1] * mom[2] - r[2] * mom[1];
        v[4] += r[2] * mom[0] - r[0] * mom[2];
        v[5] += r[0] * mom[1] - r[1] * mom[0];
    }
    // one wavefront per uncovered site: lane l < 18 takes the neighbour along
    // c_(l+1), the densities are summed over the wavefront in a fixed order,
    // lanes 0..37 write the 2 x 19 new populations
    const double sumrinit = P.rho_init[0] + P.rho_init[1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int fallback = 0;
    for (int k = wave; k < nu; k += BLOCK / 64) {
        const long long n = D.unc[off + k];
        int x, y, z;
        site_xyz(n, P, x, y, z);
        double rn[2] = {0.0, 0.0};
        bool use = false;
        if (lane < Q - 1) {
            const int i = lane + 1;
            const int mx = wrapc(x + cx(i), P.nx), my = wrapc(y + cy(i), P.ny), mz = wrapc(z + cz(i), P.nz);
            const long long m = site_of(mx, my, mz, P);
            use = owner[m] == OWN_FLUID && stage[m] == STAGE_NONE;
            if (use) {
                double r0 = 0.0, r1 = 0.0;
                for (int q = 0; q < Q; ++q) {
                    const long long src =
                        site_of(wrapc(mx - cx(q), P.nx), wrapc(my - cy(q), P.ny), wrapc(mz - cz(q), P.nz), P);
                    const auto d2 = load_pop(f, pidx(0, q, (unsigned)src));
                    r0 += (double)d2.x;
                    r1 += (double)d2.y;
                }
                rn[0] = r0 + P.rho_ref[0];
                rn[1] = r1 + P.rho_ref[1];
            }
        }
        const int cnt = __popcll(__ballot(use));
        for (int c = 0; c < 2; ++c) {
            for (int o = 32; o > 0; o >>= 1) rn[c] += __shfl_down(rn[c], o, 64);
            rn[c] = __shfl(rn[c], 0, 64);
        }
        double rnew[2];
        for (int c = 0; c < 2; ++c) {
            rnew[c] = cnt > 0 ? rn[c] / cnt : P.rho_init[c];
            if (P.c0 != 0.0 && P.rho_init[c] > 0.0) {
                const double dM = st->Mstep[c] - st->M0[c];
                rnew[c] *= 1.0 - P.c0 * (sumrinit / P.rho_init[c]) * dM / (double)N;
            }
        }
        const double r[3] = {minimg(x - R[0], L[0]), minimg(y - R[1], L[1]), minimg(z - R[2], L[2])};
        const double us[3] = {U[0] + (W[1] * r[2] - W[2] * r[1]), U[1] + (W[2] * r[0] - W[0] * r[2]),
                              U[2] + (W[0] * r[1] - W[1] * r[0])};
        const double u2 = us[0] * us[0] + us[1] * us[1] + us[2] * us[2];
        if (lane < Q) {
            // written where the site reads it: slot (i, y - c_i), read by nobody else
            const int i = lane;
            const long long dst = site_of(wrapc(x - cx(i), P.nx), wrapc(y - cy(i), P.ny), wrapc(z - cz(i), P.nz), P);
            using T = Cmp<S>;
            store_pop(f, pidx(0, i, (unsigned)dst),
                      (T)(feq_dir<double>(i, rnew[0], us[0], us[1], us[2], u2, P.eq_order) - zeta(i) * P.rho_ref[0]),
                      (T)(feq_dir<double>(i, rnew[1], us[0], us[1], us[2], u2, P.eq_order) - zeta(i) * P.rho_ref[1]));
        }
        if (lane == 0) {
            if (cnt == 0) ++fallback;
            double mom[3];
            for (int a = 0; a < 3; ++a) mom[a] = (rnew[0] + rnew[1]) * us[a];
            for (int a = 0; a < 3; ++a) v[a] -= mom[a];
            v[3] -= r[1] * mom[2] - r[2] * mom[1];
            v[4] -= r[2] * mom[0] - r[0] * mom[2];
            v[5] -= r[0] * mom[1] - r[1] * mom[0];
        }
    }
    __shared__ int nfall;
    if (threadIdx.x == 0) nfall = 0;
    __syncthreads();
    if (fallback) atomicAdd(&nfall, fallback);  // LDS, integer
    block_sum<6>(v, lds);
    if (threadIdx.x == 0) {
        for (int a = 0; a < 3; ++a) {
            D.P[3 * p + a] += v[a];
            D.PT[3 * p + a] += v[3 + a];
        }
        // the sphere's own running counts (one writer, no atomics on a
        // shared counter); k_fold_events moves them into the totals
        D.evtot[3 * p] += (unsigned long long)nc;
        D.evtot[3 * p + 1] += (unsigned long long)nu;
        D.evtot[3 * p + 2] += (unsigned long long)nfall;
    }
}

// Registers capped for 8 waves per SIMD: a sphere's block waits on a few
// dependent loads, so more resident blocks beat the 17 registers spilled
// (256^3 at a developed state: 92 -> 84 us per step, same box)
template <typename S>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8))) void k_cover_refill(DevParams P, DevParticles D, S *__restrict__ f,
                                                        const int32_t *__restrict__ owner,
                                                        const int32_t *__restrict__ stage, DevState *st) {
    cover_refill_body<S>(P, D, f, owner, stage, st, own_grid());
}

// the spheres' running event counts added to the totals, and cleared (one
// block; integer sums)
__global__ __launch_bounds__(BLOCK) void k_fold_events(DevParticles D, int np, DevState *st) {
    __shared__ unsigned long long red[3][BLOCK];
    unsigned long long c[3] = {0, 0, 0};
    for (int p = threadIdx.x; p < np; p += BLOCK)
        for (int k = 0; k < 3; ++k) {
            c[k] += D.evtot[3 * p + k];
            D.evtot[3 * p + k] = 0;
        }
    for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = c[k];
    __syncthreads();
    for (int o = BLOCK / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->covered_total += red[0][0];
        st->uncovered_total += red[1][0];
        st->refill_fallback += red[2][0];
    }
}

void launch_fold_events(lb_handle *h) {
    if (!h->np) return;
    k_fold_events<<<1, BLOCK, 0, h->stream>>>(h->dpart, h->np, h->dstate);
    LB_HIP_CHECK(hipGetLastError());
}

// owners after a full classification: the marks of the box (identical values
// from every block)
__device__ __forceinline__ void map_commit_full_body(DevParams P, DevParticles D, int32_t *__restrict__ owner,
                                                     const int32_t *__restrict__ stage, const Grid &g) {
    const int p = g.bid;
    int lo[3], ext[3];
    union_box(P, D, p, 0, lo, ext);
    const BoxWalk bw(P, lo, ext);
    const int V = bw.size();
    for (int k = threadIdx.x; k < V; k += BLOCK) {
        int u[3], x, y, z;
        bw.site(k, P, u, x, y, z);
        const long long n = site_of(x, y, z, P);
        const int32_t s = stage[n];
        owner[n] = s == STAGE_NONE ? OWN_FLUID : s;
    }
}

__global__ __launch_bounds__(BLOCK) void k_map_commit_full(DevParams P, DevParticles D, int32_t *__restrict__ owner,
                                                           const int32_t *__restrict__ stage) {
    map_commit_full_body(P, D, owner, stage, own_grid());
}

// the new owners of the sites in p's change list (a site listed by two spheres
// gets the same value twice)
__device__ __forceinline__ void map_commit_body(DevParams P, DevParticles D, int32_t *__restrict__ owner,
                                                const int32_t *__restrict__ stage, const Grid &g) {
    const int p = g.bid;
    const int off = 2 * D.ev_off[p], n = min(D.chg_cnt[p], 2 * D.ev_cap[p]);
    for (int k = threadIdx.x; k < n; k += BLOCK) {
        const int32_t s = D.chg[off + k];
        const int32_t v = stage[s];
        owner[s] = v == STAGE_FLUID ? OWN_FLUID : v;
    }
}

__global__ __launch_bounds__(BLOCK) void k_map_commit(DevParams P, DevParticles D, int32_t *__restrict__ owner,
                                                      const int32_t *__restrict__ stage) {
    map_commit_body(P, D, owner, stage, own_grid());
}

// the class words of the changed sites and their 18 neighbours (the words
// that read a changed owner), the coarse cells they lie in marked dirty; the
// change marks in stage[] are cleared
__device__ __forceinline__ void map_info_body(DevParams P, DevParticles D, const int32_t *__restrict__ owner,
                                              uint32_t *__restrict__ info, int32_t *__restrict__ stage,
                                              const Grid &g) {
    const int p = g.bid;
    const int off = 2 * D.ev_off[p], n = min(D.chg_cnt[p], 2 * D.ev_cap[p]);
    for (int k = threadIdx.x; k < n * Q; k += BLOCK) {
        const int e = k / Q, i = k - e * Q;
        const long long s = D.chg[off + e];
        int x, y, z;
        site_xyz(s, P, x, y, z);
        const int xx = wrapc(x + cx(i), P.nx), yy = wrapc(y + cy(i), P.ny), zz = wrapc(z + cz(i), P.nz);
        const long long m = site_of(xx, yy, zz, P);
        info[m] = compute_info_at(m, xx, yy, zz, P, owner) | INFO_FLAG;
        D.dirty[cell_of(D, xx, yy, zz)] = 1;
    }
    for (int k = threadIdx.x; k < n; k += BLOCK) stage[D.chg[off + k]] = STAGE_NONE;
}

__global__ __launch_bounds__(BLOCK) void k_map_info(DevParams P, DevParticles D, const int32_t *__restrict__ owner,
                                                    uint32_t *__restrict__ info, int32_t *__restrict__ stage) {
    map_info_body(P, D, owner, info, stage, own_grid());
}

constexpr int LIST_ROWS = 1024;  // box rows of the banded list walk (larger boxes scan whole)

// virtual-fluid sites of sphere p on the new map, in scan order of its box,
// and the number of its bounce-back links (fluid neighbours of those sites)
__device__ __forceinline__ void build_lists_body(DevParams P, DevParticles D, const int32_t *__restrict__ owner,
                                                       const uint32_t *__restrict__ info, DevState *st, int full, const Grid &g) {
    __shared__ int lds[8];
    __shared__ int nlink_block;
    __shared__ AxisCells ac;
    const int p = g.bid;
    if (threadIdx.x == 0) nlink_block = 0;
    int lo[3], ext[3];
    new_box(P, D, p, lo, ext);
    int32_t *lb = D.lbox + 6 * p;
    if (!full) {
        // the lists are the box scan of the class words within one site of the
        // box; when none of them changed this step and the box is the one of
        // the last build, the lists stand (and equal a rebuild)
        const bool same = lo[0] == lb[0] && lo[1] == lb[1] && lo[2] == lb[2] && ext[0] == lb[3] &&
                          ext[1] == lb[4] && ext[2] == lb[5];
        if (threadIdx.x == 0) axis_cells(P, lo, ext, ac);
        __syncthreads();
        if (!any_dirty(D, ac) && same) return;  // `same` is uniform over the block
    }
    if (threadIdx.x < 3) {
        lb[threadIdx.x] = lo[threadIdx.x];
        lb[3 + threadIdx.x] = ext[threadIdx.x];
    }
    const int soff = D.shell_off[p], scap = D.shell_cap[p];
    int nshell = 0, nlink = 0;
    const int nrow = ext[1] * ext[2];
    if (nrow <= LIST_ROWS) {
        // Only sites with r - 1.5 < |x - R| < r + 0.01 can qualify: a site of p
        // lies inside p, and a fluid neighbour (at most sqrt(2) away) lies
        // outside it.  In each box row (y, z) they form at most two x ranges
        // (rounded outwards); the walk visits them in the box's scan order, so
        // the list is the one a scan of the whole box gives.
        __shared__ int roff[LIST_ROWS + 1];
        __shared__ short rx[LIST_ROWS][4];  // [rx0, rx1) and [rx2, rx3), relative to lo[0]
        long long cq[3];
        for (int a = 0; a < 3; ++a) cq[a] = fixed20(D.R[3 * p + a]);
        const double S = 1048576.0;
        const double rq = (double)fixed20(D.rad[p]);
        const double ro = rq + 0.01 * S, ri = fmax(0.0, rq - 1.5 * S);
        const double xc = (double)cq[0] / S;
        const int per = (nrow + BLOCK - 1) / BLOCK;
        int cnt = 0;
        for (int j = 0; j < per; ++j) {
            const int r = (int)threadIdx.x * per + j;
            if (r >= nrow) break;
            const long long uy = lo[1] + r % ext[1], uz = lo[2] + r / ext[1];
            const double dy = (double)((uy << 20) - cq[1]), dz = (double)((uz << 20) - cq[2]);
            const double h2 = dy * dy + dz * dz;
            int a0 = 0, a1 = 0, b0 = 0, b1 = 0;
            if (h2 < ro * ro) {
                const double xa = sqrt(ro * ro - h2) / S, xb = h2 < ri * ri ? sqrt(ri * ri - h2) / S : 0.0;
                int l0 = (int)floor(xc - xa), l1 = (int)ceil(xc - xb) + 1;
                int r0 = (int)floor(xc + xb), r1 = (int)ceil(xc + xa) + 1;
                if (l1 >= r0) {  // one range
                    l1 = r1;
                    r0 = r1;
                }
                const int e0 = lo[0], e1 = lo[0] + ext[0];
                l0 = max(l0, e0);
                l1 = max(min(l1, e1), l0);
                r0 = max(r0, l1);
                r1 = max(min(r1, e1), r0);
                a0 = l0 - e0;
                a1 = l1 - e0;
                b0 = r0 - e0;
                b1 = r1 - e0;
            }
            rx[r][0] = (short)a0;
            rx[r][1] = (short)a1;
            rx[r][2] = (short)b0;
            rx[r][3] = (short)b1;
            cnt += (a1 - a0) + (b1 - b0);
        }
        int tot;
        int base = block_scan_excl(cnt, tot, lds);  // barrier: every rx row is written
        for (int j = 0; j < per; ++j) {
            const int r = (int)threadIdx.x * per + j;
            if (r >= nrow) break;
            roff[r] = base;
            base += (rx[r][1] - rx[r][0]) + (rx[r][3] - rx[r][2]);
        }
        if (threadIdx.x == 0) roff[nrow] = tot;
        __syncthreads();
        for (int start = 0; start < tot; start += BLOCK) {
            const int k = start + threadIdx.x;
            bool sh = false;
            long long n = 0;
            if (k < tot) {
                int rl = 0, rh = nrow;  // roff[rl] <= k < roff[rh]
                while (rh - rl > 1) {
                    const int mid = (rl + rh) >> 1;
                    if (roff[mid] <= k) rl = mid;
                    else rh = mid;
                }
                const int off = k - roff[rl], la = rx[rl][1] - rx[rl][0];
                const int dx = off < la ? rx[rl][0] + off : rx[rl][2] + (off - la);
                const int x = wrapany(lo[0] + dx, P.nx), y = wrapany(lo[1] + rl % ext[1], P.ny),
                          z = wrapany(lo[2] + rl / ext[1], P.nz);
                n = site_of(x, y, z, P);
                const uint32_t inf = info[n];
                sh = owner[n] == p && site_class(inf) == CLS_SHELL;
                if (sh) nlink += __popc(~inf & 0x7fffeu);
            }
            const int slot = block_compact(sh, nshell, lds);
            if (sh && slot < scap) D.shell[soff + slot] = (int32_t)n;
        }
    } else {
        const BoxWalk bw(P, lo, ext);
        const int V = bw.size();
        for (int start = 0; start < V; start += BLOCK) {
            const int k = start + threadIdx.x;
            bool sh = false;
            long long n = 0;
            if (k < V) {
                int u[3], x, y, z;
                bw.site(k, P, u, x, y, z);
                n = site_of(x, y, z, P);
                const uint32_t inf = info[n];
                sh = owner[n] == p && site_class(inf) == CLS_SHELL;
                if (sh) nlink += __popc(~inf & 0x7fffeu);
            }
            const int slot = block_compact(sh, nshell, lds);
            if (sh && slot < scap) D.shell[soff + slot] = (int32_t)n;
        }
    }
    atomicAdd(&nlink_block, nlink);  // integer sum: order does not matter
    __syncthreads();
    if (threadIdx.x == 0) {
        D.shell_cnt[p] = nshell;
        D.link_cnt[p] = nlink_block;
        if (nshell > scap) atomicOr(&st->overflow, 2);
    }
}

__global__ __launch_bounds__(BLOCK) void k_build_lists(DevParams P, DevParticles D, const int32_t *__restrict__ owner,
                                                       const uint32_t *__restrict__ info, DevState *st, int full) {
    build_lists_body(P, D, owner, info, st, full, own_grid());
}

// ---------------------------------------------------------------------------
// launchers (one block per sphere unless noted)
// ---------------------------------------------------------------------------
void launch_particle_fluid_force(lb_handle *h, void *fout) {
    if (!h->np) return;
    with_storage(h->prm, [&](auto tag) {
        using S = typename decltype(tag)::type;
        using T = Cmp<S>;
        k_particle_fluid_force<S><<<h->np, BLOCK, 0, h->stream>>>(h->dp, h->dpart, (S *)fout, (const T *)h->rho,
                                                                  (const T *)h->fsc, h->info);
    });
    LB_HIP_CHECK(hipGetLastError());
}

// the cell list (PAIR_CELLS_MIN_SPHERES) pays off from about a thousand
// spheres; fewer take the all-pairs kernel (one launch instead of four)
void launch_pair_forces(lb_handle *h, hipStream_t s) {
    if (!h->np) return;
    if (h->dpart.pgx > 0 && h->np >= PAIR_CELLS_MIN_SPHERES) {
        const unsigned nb = (unsigned)((h->np + BLOCK - 1) / BLOCK);
        k_pcell_count<<<nb, BLOCK, 0, s>>>(h->dp, h->dpart);
        k_pcell_scan<<<1, PCS_THREADS, 0, s>>>(h->dpart);
        k_pcell_fill<<<nb, BLOCK, 0, s>>>(h->dp, h->dpart);
        k_pair_forces_cells<<<h->np, 64, 0, s>>>(h->dp, h->dpart, h->dstate);
    } else {
        k_pair_forces<<<h->np, BLOCK, 0, s>>>(h->dp, h->dpart, h->dstate);
    }
    LB_HIP_CHECK(hipGetLastError());
}

void launch_forces_total(lb_handle *h) {
    if (!h->np) return;
    k_forces_total<<<(h->np + BLOCK - 1) / BLOCK, BLOCK, 0, h->stream>>>(h->dp, h->dpart);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_integrate(lb_handle *h) {
    if (!h->np) return;
    k_integrate<<<(h->np + BLOCK - 1) / BLOCK, BLOCK, 0, h->stream>>>(h->dp, h->dpart, h->dstate);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_map_mark(lb_handle *h) {
    if (!h->np) return;
    k_map_mark<<<h->np, BLOCK, 0, h->stream>>>(h->dp, h->dpart, h->stage);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_map_flip(lb_handle *h) {
    if (!h->np) return;
    k_map_flip<<<h->np, BLOCK, 0, h->stream>>>(h->dp, h->dpart, h->owner, h->stage, h->info, h->dstate);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_map_fixup(lb_handle *h, void *fout) {
    if (!h->np) return;
    with_storage(h->prm, [&](auto tag) {
        using S = typename decltype(tag)::type;
        using T = Cmp<S>;
        k_map_fixup<S><<<h->np, BLOCK, 0, h->stream>>>(h->dp, h->dpart, (S *)fout, (const T *)h->rho, h->owner,
                                                       h->info);
    });
    LB_HIP_CHECK(hipGetLastError());
}

void launch_materialize(lb_handle *h, void *f) {
    if (!h->np) return;
    with_storage(h->prm, [&](auto tag) {
        using S = typename decltype(tag)::type;
        using T = Cmp<S>;
        k_materialize<S><<<(unsigned)((h->N + BLOCK - 1) / BLOCK), BLOCK, 0, h->stream>>>(h->dp, h->dpart, (S *)f, (const T *)h->rho, h->owner,
                                                              h->info);
    });
    LB_HIP_CHECK(hipGetLastError());
}

void launch_cover_refill(lb_handle *h, void *fout) {
    if (!h->np) return;
    with_storage(h->prm, [&](auto tag) {
        using S = typename decltype(tag)::type;
        k_cover_refill<S><<<h->np, BLOCK, 0, h->stream>>>(h->dp, h->dpart, (S *)fout, h->owner, h->stage, h->dstate);
    });
    LB_HIP_CHECK(hipGetLastError());
}

void launch_map_commit(lb_handle *h, bool full) {
    if (!h->np) return;
    if (full)
        k_map_commit_full<<<h->np, BLOCK, 0, h->stream>>>(h->dp, h->dpart, h->owner, h->stage);
    else
        k_map_commit<<<h->np, BLOCK, 0, h->stream>>>(h->dp, h->dpart, h->owner, h->stage);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_map_info(lb_handle *h) {
    if (!h->np) return;
    k_map_info<<<h->np, BLOCK, 0, h->stream>>>(h->dp, h->dpart, h->owner, h->info, h->stage);
    LB_HIP_CHECK(hipGetLastError());
}

void launch_build_lists(lb_handle *h, bool full, hipStream_t s) {
    if (!h->np) return;
    k_build_lists<<<h->np, BLOCK, 0, s>>>(h->dp, h->dpart, h->owner, h->info, h->dstate, full ? 1 : 0);
    LB_HIP_CHECK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Batched launches: each block finds its member and its place in the member's
// range and runs the same body as the single-lattice kernel, so every member
// computes exactly what it computes alone.
// ---------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(BLOCK) void kb_particle_fluid_force(BatchPlan B) {
    using T = Cmp<S>;
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_SPHERE, g)];
    particle_fluid_force_body<S>(M.P, M.D, (S *)M.fout, (const T *)M.rho, (const T *)M.fsc, M.info, g);
}
__global__ void kb_pcell_count(BatchPlan B) {
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_CELL_SPH256, g)];
    pcell_count_body(M.P, M.D, g);
}
__global__ __launch_bounds__(PCS_THREADS) void kb_pcell_scan(BatchPlan B) {
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_CELL_ONE, g)];
    pcell_scan_body(M.D, g);
}
__global__ void kb_pcell_fill(BatchPlan B) {
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_CELL_SPH256, g)];
    pcell_fill_body(M.P, M.D, g);
}
__global__ __launch_bounds__(64) void kb_pair_forces_cells(BatchPlan B) {
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_CELL_SPHERE, g)];
    pair_forces_cells_body(M.P, M.D, M.dstate, g);
}
__global__ __launch_bounds__(BLOCK) void kb_pair_forces(BatchPlan B) {
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_PAIR_SPHERE, g)];
    pair_forces_body(M.P, M.D, M.dstate, g);
}
__global__ void kb_forces_total(BatchPlan B) {
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_SPHERE256, g)];
    forces_total_body(M.P, M.D, g);
}
__global__ void kb_integrate(BatchPlan B) {
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_SPHERE256, g)];
    integrate_body(M.P, M.D, M.dstate, g);
}
__global__ __launch_bounds__(BLOCK) void kb_map_flip(BatchPlan B) {
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_SPHERE, g)];
    map_flip_body(M.P, M.D, M.owner, M.stage, M.info, M.dstate, g);
}
template <typename S>
__global__ __launch_bounds__(BLOCK) void kb_cover_refill(BatchPlan B) {
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_SPHERE, g)];
    cover_refill_body<S>(M.P, M.D, (S *)M.fout, M.owner, M.stage, M.dstate, g);
}
__global__ __launch_bounds__(BLOCK) void kb_map_commit(BatchPlan B) {
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_SPHERE, g)];
    map_commit_body(M.P, M.D, M.owner, M.stage, g);
}
__global__ __launch_bounds__(BLOCK) void kb_map_info(BatchPlan B) {
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_SPHERE, g)];
    map_info_body(M.P, M.D, M.owner, M.info, M.stage, g);
}
__global__ __launch_bounds__(BLOCK) void kb_build_lists(BatchPlan B) {
    Grid g;
    const BatchMember &M = B.m[batch_member(B, BM_SPHERE, g)];
    build_lists_body(M.P, M.D, M.owner, M.info, M.dstate, 0, g);
}

// the particle stages of one step of every member, in the order of a single
// lattice's step (link sums, pair search, integration, map update)
void launch_batch_particles(const BatchLaunch &L, int parity, hipStream_t s) {
    const BatchPlan &B = L.plan[parity];
    const unsigned nsph = (unsigned)L.total[BM_SPHERE];
    if (nsph == 0) return;
    with_storage(L.prm, [&](auto tag) {
        using S = typename decltype(tag)::type;
        kb_particle_fluid_force<S><<<nsph, BLOCK, 0, s>>>(B);
    });
    if (L.total[BM_CELL_SPHERE] > 0) {
        kb_pcell_count<<<(unsigned)L.total[BM_CELL_SPH256], BLOCK, 0, s>>>(B);
        kb_pcell_scan<<<(unsigned)L.total[BM_CELL_ONE], PCS_THREADS, 0, s>>>(B);
        kb_pcell_fill<<<(unsigned)L.total[BM_CELL_SPH256], BLOCK, 0, s>>>(B);
        kb_pair_forces_cells<<<(unsigned)L.total[BM_CELL_SPHERE], 64, 0, s>>>(B);
    }
    if (L.total[BM_PAIR_SPHERE] > 0) kb_pair_forces<<<(unsigned)L.total[BM_PAIR_SPHERE], BLOCK, 0, s>>>(B);
    kb_forces_total<<<(unsigned)L.total[BM_SPHERE256], BLOCK, 0, s>>>(B);
    kb_integrate<<<(unsigned)L.total[BM_SPHERE256], BLOCK, 0, s>>>(B);
    kb_map_flip<<<nsph, BLOCK, 0, s>>>(B);
    with_storage(L.prm, [&](auto tag) {
        using S = typename decltype(tag)::type;
        kb_cover_refill<S><<<nsph, BLOCK, 0, s>>>(B);
    });
    kb_map_commit<<<nsph, BLOCK, 0, s>>>(B);
    kb_map_info<<<nsph, BLOCK, 0, s>>>(B);
    kb_build_lists<<<nsph, BLOCK, 0, s>>>(B);
    LB_HIP_CHECK(hipGetLastError());
}

}  // namespace lbm
