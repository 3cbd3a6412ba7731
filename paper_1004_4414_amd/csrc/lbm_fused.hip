// Single-sweep fluid step for gfx950: densities, virtual fluid, Shan-Chen
// force, collision with the velocity shift and pull streaming for one time
// step (Secs. II-IV of Jansen & Harting) in one kernel that reads each
// population from HBM once and writes it once.
//
// A workgroup owns a 64 x TY column of sites (one wavefront per row) and
// marches in z over a segment of planes.  Per plane zc it runs three stages
// separated by barriers; all global loads of an iteration are issued in stage
// A, before any of them is waited for:
//   A: every thread pulls the 19 populations of both components of its own
//      site in plane zc+1 into registers (kept until the next iteration, when
//      the site is collided: nothing is read twice) and stores the site's
//      density deviation in an LDS ring.  Two wavefronts add the pull sums of
//      the one-site halo's rows below and above the tile (whole rows, with
//      the row addressing of the own pulls); the work list built in stage B
//      of the previous iteration adds those of its two columns (fluid sites
//      without a solid neighbour) and of the fluid sites of plane zc+2
//      (two-site halo) that have one, the only fluid sites a virtual-fluid
//      average reads.  The class words of plane zc+3 (two-site halo) go into
//      a four-plane LDS ring, so that every list is known one iteration
//      ahead.
//   B (plane zc+1): Psi - Psi(rho_ref) of the tile and the one-site halo:
//      fluid sites from their density, virtual-fluid sites from the mean
//      density of their fluid neighbours in planes zc..zc+2 plus the colour
//      (Sec. IV, Eqs. (27), (29), (30)), other solid sites Psi = 0 (Eq. (5)).
//      Then the work list of the next iteration.
//   C (plane zc): each thread forms the Shan-Chen force of Eq. (4) from the
//      Psi ring and collides its site from the registers filled one plane
//      earlier (Eqs. (2), (3), (6)); it stores f* in its own slots (zeros on
//      non-fluid sites, the Shan-Chen force of a virtual-fluid site in that
//      site's slots).  The link kernels bounce the populations at solid
//      neighbours afterwards, as for the two-pass sweep.
// The halo is recomputed rather than exchanged, so no workgroup waits for
// another; workgroups that share an XCD are spatial neighbours, which keeps
// the halo pulls in that XCD's L2.  Each site's density is summed in the same
// order as the two-pass density sweep, so the two variants compute the same
// values.
#include "lbm_handle.h"

namespace lbm {

// Tuning macro (compile time): LBM_FUSED_STREAM = 1 puts the streaming hint
// on the own pulls that no other wavefront of the tile reads, as the two-pass
// sweep does; 0 leaves them in the caches for the halo pulls of neighbouring
// tiles.
#ifndef LBM_FUSED_STREAM
#define LBM_FUSED_STREAM 0
#endif

constexpr int FTX = 64;                // tile width: one wavefront per row
constexpr uint32_t LINK_BITS = 0x7fffeu;  // bits 1..18 of a class word

template <typename T, int TY>
struct FusedLds {
    static constexpr int NT = FTX * TY;                                 // threads
    static constexpr int R2X = FTX + 4, R2Y = TY + 4, R2N = R2X * R2Y;  // tile + two-site halo
    static constexpr int R1X = FTX + 2, R1Y = TY + 2, R1N = R1X * R1Y;  // tile + one-site halo
    static constexpr int NRING1 = R1N - NT;                             // the one-site halo alone
    static constexpr int LMAX = NRING1 + R2N;                           // longest work list
    static constexpr int CW = (R2N + NT - 1) / NT;                      // class words per thread
    T rho[3][2][R2N];         // density deviations, planes mod 3
    uint32_t cls[4][R2N];     // class words, planes mod 4
    T psi[3][2][R1N];         // Psi - Psi(rho_ref), planes mod 3
    T col[R1N];               // colours of the virtual-fluid sites of the plane in stage B
    uint16_t item[2][LMAX];   // pull-sum work lists (cell | 0x8000 for the plane two ahead)
    int count[2];             // their lengths
    int xw[R2X], yw[R2Y];     // the region's columns and rows, wrapped into the box
    double red[2 * NT / 64];
};

__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb) {
    // hardware dispatches block b to XCD b % 8; give each XCD a contiguous range
    if (nb % 8u) return b;
    return (b % 8u) * (nb / 8u) + b / 8u;
}
__device__ __forceinline__ int mod3(int a) { return ((a % 3) + 3) % 3; }
__device__ __forceinline__ int mod4(int a) { return a & 3; }

template <typename S, typename M, int TY, bool ROWS>
__global__ __launch_bounds__(FTX *TY) void k_fused_step(DevParams P, DevParticles D, const S *__restrict__ fin,
                                                        S *__restrict__ fout, Cmp<S> *__restrict__ rho_out,
                                                        const uint32_t *__restrict__ info,
                                                        const int32_t *__restrict__ owner, Cmp<S> *__restrict__ fsc,
                                                        double *__restrict__ partial, int TZ, int ntx, int nty) {
    using T = Cmp<S>;
    using L = FusedLds<T, TY>;
    __shared__ L sm;
    const int t = threadIdx.x;
    const unsigned blk = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = (int)(blk % (unsigned)(ntx * nty));
    const int seg = (int)(blk / (unsigned)(ntx * nty));
    const int x0 = (tile % ntx) * FTX, y0 = (tile / ntx) * TY, z0 = seg * TZ;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int zend = min(z0 + TZ, nz);
    const T irho0 = (T)P.inv_rho0;
    const T e0 = (T)P.psi_e[0], e1 = (T)P.psi_e[1];
    // Psi - Psi(rho_ref) of a site without fluid (Psi = 0)
    const T psolid0 = psi_dev(-(T)P.rho_ref[0], e0, irho0), psolid1 = psi_dev(-(T)P.rho_ref[1], e1, irho0);
    double mass0 = 0.0, mass1 = 0.0;

    // this thread's own site (collided in stage C)
    const int tx = t % FTX, ty = t / FTX;
    const int xs = x0 + tx, ys = y0 + ty;
    const bool mine = xs < nx && ys < ny;
    const int own2 = (ty + 2) * L::R2X + tx + 2;
    const int own1 = (ty + 1) * L::R1X + tx + 1;
    // the own cell past the box edge of a ragged tile stands for its periodic image
    const int xo = wrapany(xs, nx), yo = wrapany(ys, ny);

    // the region's wrapped coordinates, and the class-word cells of this thread
    for (int s = t; s < L::R2X; s += L::NT) sm.xw[s] = wrapany(x0 - 2 + s, nx);
    for (int s = t; s < L::R2Y; s += L::NT) sm.yw[s] = wrapany(y0 - 2 + s, ny);
    int cwo[L::CW];  // in-plane site offsets of the class-word cells (-1: none)
#pragma unroll
    for (int j = 0; j < L::CW; ++j) {
        const int s = t + j * L::NT;
        cwo[j] = s < L::R2N ? wrapany(y0 - 2 + s / L::R2X, ny) * nx + wrapany(x0 - 2 + s % L::R2X, nx) : -1;
    }
    // halo rows: wavefront 0 the row below the tile, wavefront 1 the row above
    const int lane = t & 63, wave = t >> 6;
    const bool hrow = wave < 2;
    const int hy = wrapany(wave == 0 ? y0 - 1 : y0 + TY, ny), hx = wrapany(x0 + lane, nx);
    const int hs2 = (wave == 0 ? 1 : TY + 2) * L::R2X + lane + 2;
    const long long nxy = (long long)nx * ny;

    T cur[2][Q], nxt[2][Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) cur[0][i] = cur[1][i] = nxt[0][i] = nxt[1][i] = (T)0;
    uint32_t cur_inf = 0;
    if (t < 2) sm.count[t] = 0;
    __syncthreads();

    for (int zc = z0 - 5; zc < zend; ++zc) {
        // ---------------- stage A: issue every load of the iteration ----------------
        const int za = zc + 1;
        const int zwa = wrapany(za, nz);
        const int sla = mod3(za);
        const bool live = za >= z0 - 1;  // plane zc+1 feeds a Psi that a collision reads
        // class words of plane zc+3 over the two-site halo
        uint32_t cw[L::CW];
        {
            const long long zo = (long long)wrapany(zc + 3, nz) * nxy;
#pragma unroll
            for (int j = 0; j < L::CW; ++j) cw[j] = cwo[j] >= 0 ? info[zo + cwo[j]] : 0u;
        }
        // colours of the virtual-fluid sites of plane zc+1 (coloured spheres only)
        constexpr int CC = (L::R1N + L::NT - 1) / L::NT;
        double colv[CC];
        if (P.any_color && live) {
#pragma unroll
            for (int j = 0; j < CC; ++j) {
                const int s = t + j * L::NT;
                colv[j] = 0.0;
                if (s < L::R1N) {
                    const int bx = s % L::R1X, by = s / L::R1X;
                    if (site_class(sm.cls[mod4(za)][(by + 1) * L::R2X + bx + 1]) == CLS_SHELL)
                        colv[j] = D.color[owner[zwa * nxy + (long long)sm.yw[by + 1] * nx + sm.xw[bx + 1]]];
                }
            }
        }
        // the own site of plane zc+1
        if (live) {
            const bool own_fluid = site_class(sm.cls[mod4(za)][own2]) == CLS_FLUID;
            if (own_fluid) {
                T d0 = 0, d1 = 0;
                if (mine && za >= z0 && za < zend) {  // collided at the next iteration: keep the pulls
                    if constexpr (ROWS) {
                        const RowView<S> rv(P, xs, ys, zwa);
                        pull_load_rows<S, LBM_FUSED_STREAM != 0>(fin, rv, nxt);
                    } else {
                        pull_load(fin, (unsigned)(zwa * nxy + (long long)ys * nx + xs), NbrOffsets(P, xs, ys, zwa), nxt);
                    }
                    Unroll<Q>::run([&](auto ic) {
                        constexpr int i = decltype(ic)::value;
                        d0 += nxt[0][i];
                        d1 += nxt[1][i];
                    });
                } else {
                    pull_sum(fin, (unsigned)(zwa * nxy + (long long)yo * nx + xo), NbrOffsets(P, xo, yo, zwa), d0, d1);
                }
                sm.rho[sla][0][own2] = d0;
                sm.rho[sla][1][own2] = d1;
            }
            // the halo rows below and above the tile
            if (hrow && site_class(sm.cls[mod4(za)][hs2]) == CLS_FLUID) {
                T d0, d1;
                if constexpr (ROWS) {
                    const RowView<S> rv(P, hx, hy, zwa);
                    pull_sum_rows<S, false>(fin, rv, d0, d1);
                } else {
                    pull_sum(fin, (unsigned)(zwa * nxy + (long long)hy * nx + hx), NbrOffsets(P, hx, hy, zwa), d0, d1);
                }
                sm.rho[sla][0][hs2] = d0;
                sm.rho[sla][1][hs2] = d1;
            }
        }
        // the work list: halo columns of plane zc+1, boundary sites of plane zc+2
        {
            const int nitem = sm.count[zc & 1];
            constexpr int IT0 = 2 * 64;  // the two halo-row wavefronts take no items
            for (int j = t - IT0; j < nitem; j += L::NT - IT0) {
                if (j < 0) break;
                const uint32_t e = sm.item[zc & 1][j];
                const int cell = (int)(e & 0x7fffu);
                const int zp = e & 0x8000u ? zc + 2 : zc + 1;
                const int x = sm.xw[cell % L::R2X], y = sm.yw[cell / L::R2X];
                const int zw = wrapany(zp, nz);
                T s0, s1;
                pull_sum(fin, (unsigned)(zw * nxy + (long long)y * nx + x), NbrOffsets(P, x, y, zw), s0, s1);
                sm.rho[mod3(zp)][0][cell] = s0;
                sm.rho[mod3(zp)][1][cell] = s1;
            }
        }
#pragma unroll
        for (int j = 0; j < L::CW; ++j) {
            const int s = t + j * L::NT;
            if (s < L::R2N) sm.cls[mod4(zc + 3)][s] = cw[j];
        }
        if (P.any_color && live) {
#pragma unroll
            for (int j = 0; j < CC; ++j) {
                const int s = t + j * L::NT;
                if (s < L::R1N) sm.col[s] = (T)colv[j];
            }
        }
        if (t == 0) sm.count[(zc + 1) & 1] = 0;  // the list that stage B fills
        __syncthreads();
        // ---------------- stage B, plane zc+1: Psi of the tile and its one-site halo ----------------
        if (za >= z0 - 1) {
            const int slm = mod3(za - 1), sl0 = mod3(za), slp = mod3(za + 1);
            for (int s = t; s < L::R1N; s += L::NT) {
                const int bx = s % L::R1X, by = s / L::R1X;
                const int s2 = (by + 1) * L::R2X + bx + 1;
                const uint32_t inf = sm.cls[mod4(za)][s2];
                const uint32_t cls = site_class(inf);
                T p0 = psolid0, p1 = psolid1;
                if (cls == CLS_FLUID) {
                    p0 = psi_dev(sm.rho[sl0][0][s2], e0, irho0);
                    p1 = psi_dev(sm.rho[sl0][1][s2], e1, irho0);
                } else if (cls == CLS_SHELL) {
                    // the class word of a virtual-fluid site flags its non-fluid
                    // neighbours; the others are summed in direction order
                    T s0 = 0, s1 = 0;
                    int nf = 0;
#pragma unroll
                    for (int i = 1; i < Q; ++i) {
                        const int sl = cz(i) < 0 ? slm : (cz(i) > 0 ? slp : sl0);
                        const int sn = s2 + cy(i) * L::R2X + cx(i);
                        const bool fl = !((inf >> i) & 1u);
                        const T a0 = sm.rho[sl][0][sn], a1 = sm.rho[sl][1][sn];
                        s0 += fl ? a0 : (T)0;
                        s1 += fl ? a1 : (T)0;
                        nf += fl;
                    }
                    T r0 = nf ? s0 / (T)nf : (T)0, r1 = nf ? s1 / (T)nf : (T)0;
                    if (P.any_color) {
                        const T col = sm.col[s];
                        if (col > (T)0) r0 += fabs(col);
                        if (col < (T)0) r1 += fabs(col);
                    }
                    p0 = psi_dev(r0, e0, irho0);
                    p1 = psi_dev(r1, e1, irho0);
                }
                sm.psi[sl0][0][s] = p0;
                sm.psi[sl0][1][s] = p1;
            }
            // the own class word of plane zc, before its slot is reused
            if (zc >= z0) cur_inf = sm.cls[mod4(zc)][own2];
        }
        // the work list of the next iteration: fluid sites of the halo columns
        // of plane zc+2 without a solid neighbour, and fluid sites of plane
        // zc+3 with one
        {
            const int nl = (zc + 1) & 1;
            if (zc + 2 >= z0 - 1) {
                for (int r = t; r < 2 * (TY + 2); r += L::NT) {
                    const int bx = r < TY + 2 ? 0 : L::R1X - 1, by = r < TY + 2 ? r : r - (TY + 2);
                    const int s2 = (by + 1) * L::R2X + bx + 1;
                    const uint32_t inf = sm.cls[mod4(zc + 2)][s2];
                    if (site_class(inf) == CLS_FLUID && !(inf & LINK_BITS))
                        sm.item[nl][atomicAdd(&sm.count[nl], 1)] = (uint16_t)s2;
                }
            }
            for (int s = t; s < L::R2N; s += L::NT) {
                const uint32_t inf = sm.cls[mod4(zc + 3)][s];
                if (site_class(inf) == CLS_FLUID && (inf & LINK_BITS))
                    sm.item[nl][atomicAdd(&sm.count[nl], 1)] = (uint16_t)(s | 0x8000);
            }
        }
        __syncthreads();
        // ---------------- stage C, plane zc: force, collision, own-slot stores ----------------
        if (zc >= z0 && mine) {
            const int slm = mod3(zc - 1), sl0 = mod3(zc), slp = mod3(zc + 1);
            const uint32_t inf = cur_inf;
            const uint32_t cls = site_class(inf);
            const unsigned n = (unsigned)(((long long)zc * ny + ys) * nx + xs);
            T f[2][Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                f[0][i] = cls == CLS_FLUID ? cur[0][i] : (T)0;
                f[1][i] = cls == CLS_FLUID ? cur[1][i] : (T)0;
            }
            if (cls == CLS_FLUID || cls == CLS_SHELL) {
                T pn[2][Q - 1], acc[2][3];
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    const int sl = cz(i) < 0 ? slm : (cz(i) > 0 ? slp : sl0);
                    const int sn = own1 + cy(i) * L::R1X + cx(i);
                    pn[0][i - 1] = sm.psi[sl][0][sn];
                    pn[1][i - 1] = sm.psi[sl][1][sn];
                }
                psi_force_sum(P, pn, acc);
                if (cls == CLS_SHELL) {
                    const T own[2] = {sm.psi[sl0][0][own1], sm.psi[sl0][1][own1]};
                    T F[3];
                    shell_force(P, own, acc, F);
                    if (shell_force_in_slots<S>(inf)) {
                        put_shell_force(f, F, inf);
                    } else {
#pragma unroll
                        for (int a = 0; a < 3; ++a) fsc[vidx(a, n)] = F[a];
                    }
                } else {
                    collide_site<M>(P, f, acc, inf, n, rho_out, mass0, mass1);
                }
            }
            if constexpr (ROWS) {
                const RowView<S> rv(P, xs, ys, zc);
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
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            cur[0][i] = nxt[0][i];
            cur[1][i] = nxt[1][i];
        }
    }
    // per-block fluid mass (fixed order: lanes, then waves)
    double m[2] = {mass0, mass1};
#pragma unroll
    for (int c = 0; c < 2; ++c)
        for (int off = 32; off > 0; off >>= 1) m[c] += __shfl_down(m[c], off, 64);
    if ((t & 63) == 0) {
        sm.red[2 * (t >> 6)] = m[0];
        sm.red[2 * (t >> 6) + 1] = m[1];
    }
    __syncthreads();
    if (t == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int w = 0; w < L::NT / 64; ++w) {
            s0 += sm.red[2 * w];
            s1 += sm.red[2 * w + 1];
        }
        partial[2 * blockIdx.x] = s0;
        partial[2 * blockIdx.x + 1] = s1;
    }
}

// ---------------------------------------------------------------------------
template <typename S, int TY>
static void launch_fused_t(lb_handle *h, const void *fin, void *fout) {
    using T = Cmp<S>;
    const int ntx = (h->prm.nx + FTX - 1) / FTX, nty = (h->prm.ny + TY - 1) / TY;
    const int TZ = h->fused_tz;
    const int nseg = (h->prm.nz + TZ - 1) / TZ;
    const unsigned nb = (unsigned)(ntx * nty * nseg);
    const bool rows = h->prm.nx % FTX == 0;
    with_model(h->prm, [&](auto m) {
        using Mo = decltype(m);
        if (rows)
            k_fused_step<S, Mo, TY, true><<<nb, FTX * TY, 0, h->stream>>>(
                h->dp, h->dpart, (const S *)fin, (S *)fout, (T *)h->rho, h->info, h->owner, (T *)h->fsc, h->partial,
                TZ, ntx, nty);
        else
            k_fused_step<S, Mo, TY, false><<<nb, FTX * TY, 0, h->stream>>>(
                h->dp, h->dpart, (const S *)fin, (S *)fout, (T *)h->rho, h->info, h->owner, (T *)h->fsc, h->partial,
                TZ, ntx, nty);
    });
    LB_HIP_CHECK(hipGetLastError());
    h->n_fused_blocks = (int)nb;
}

// every box: the halo coordinates are reduced modulo the box edges
bool fused_supported(const lb_params &) { return true; }

void launch_fused(lb_handle *h, const void *fin, void *fout) {
    const int ty = h->fused_ty;
    with_storage(h->prm, [&](auto tag) {
        using S = typename decltype(tag)::type;
        if constexpr (std::is_same<S, double>::value) launch_fused_t<S, 4>(h, fin, fout);
        else if (ty == 8) launch_fused_t<S, 8>(h, fin, fout);
        else launch_fused_t<S, 4>(h, fin, fout);
    });
}

}  // namespace lbm
