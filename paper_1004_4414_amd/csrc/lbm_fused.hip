// Single-sweep fluid step for gfx950: densities, virtual fluid, Shan-Chen
// force, collision with the velocity shift and pull streaming for one time
// step (Secs. II-IV of Jansen & Harting) in one kernel that reads and writes
// each population once from HBM.
//
// A workgroup owns a TX x TY column of sites and marches in z over TZ planes.
// Per plane it runs three stages separated by barriers:
//   A (plane z+2): density deviations of the tile and a 2-site halo into an
//      LDS ring (halo sites two away only when they border a solid site: only
//      the virtual fluid reads them);
//   B (plane z+1): virtual-fluid densities of shell sites (mean over fluid
//      neighbours, planes z..z+2) and Psi - Psi(rho_ref) of the tile and a
//      1-site halo into a second LDS ring;
//   C (plane z):   each thread re-reads its site's populations (still in
//      L2 / the Infinity Cache from stage A two planes earlier), forms the
//      Shan-Chen force from the Psi ring, collides and stores f* in its own
//      slots (aligned; zeros on non-fluid sites); the link kernels bounce
//      the populations at solid neighbours afterwards.
// The halo is recomputed instead of exchanged, so no workgroup waits for
// another.  Tiles that share an XCD are spatial neighbours (blockIdx is
// remapped so each XCD walks a contiguous range of tiles), which keeps halo
// re-reads in that XCD's L2.
#include "lbm_handle.h"

namespace lbm {

template <typename T, int TX, int TY>
struct FusedShape {
    static constexpr int NT = TX * TY;              // threads
    static constexpr int AX = TX + 4, AY = TY + 4;  // stage-A region (halo 2)
    static constexpr int BX = TX + 2, BY = TY + 2;  // stage-B region (halo 1)
    static constexpr int AN = AX * AY, BN = BX * BY;
    static constexpr int RING = 4;
};

template <typename T, int TX, int TY>
struct FusedLds {
    using S = FusedShape<T, TX, TY>;
    T drho[S::RING][2][S::AN];      // density deviations (fluid), virtual densities (shell)
    uint32_t info[S::RING][S::AN];  // class words
    T psi[S::RING][2][S::BN];       // Psi - Psi(rho_ref)
    double red[2 * S::NT / 64];     // per-wave partial masses
};

__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb) {
    // hardware dispatches block b to XCD b % 8; give each XCD a contiguous range
    if (nb % 8u) return b;
    return (b % 8u) * (nb / 8u) + b / 8u;
}

template <typename T, int TX, int TY, typename M>
__global__ __launch_bounds__(TX *TY) void k_fused_step(DevParams P, DevParticles D, const T *__restrict__ fin,
                                                       T *__restrict__ fout, T *__restrict__ rho,
                                                       const uint32_t *__restrict__ info,
                                                       const int32_t *__restrict__ owner, T *__restrict__ fsc,
                                                       double *__restrict__ partial, int TZ, int ntx, int nty) {
    using S = FusedShape<T, TX, TY>;
    __shared__ FusedLds<T, TX, TY> sm;
    const int t = threadIdx.x;
    const unsigned blk = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = (int)(blk % (unsigned)(ntx * nty));
    const int seg = (int)(blk / (unsigned)(ntx * nty));
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY, z0 = seg * TZ;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const long long N = P.N;
    const int zend = min(z0 + TZ, nz);
    const T ref0 = (T)P.rho_ref[0], ref1 = (T)P.rho_ref[1];
    const T rho0 = (T)P.rho0, irho0 = (T)P.inv_rho0, g = (T)P.g;
    const T e0 = (T)P.psi_e[0], e1 = (T)P.psi_e[1];
    // Psi - Psi(rho_ref) of a site without fluid (Psi = 0)
    const T psolid0 = psi_dev(-ref0, e0, irho0), psolid1 = psi_dev(-ref1, e1, irho0);
    double mass0 = 0.0, mass1 = 0.0;

    // own site of this thread in stage C
    const int tx = t % TX, ty = t / TX;
    const int xs = x0 + tx, ys = y0 + ty;
    const bool mine = xs < nx && ys < ny;

    const int nplanes = zend - z0;
    for (int k = 0; k < nplanes + 4; ++k) {
        // ---------------- stage A: plane za = z0 - 2 + k ----------------
        {
            const int za = wrapc(z0 - 2 + k, nz);
            const int slot = (z0 - 2 + k + 8) % S::RING;
            for (int s = t; s < S::AN; s += S::NT) {
                const int ax = s % S::AX, ay = s / S::AX;
                const int x = wrapc(x0 - 2 + ax, nx), y = wrapc(y0 - 2 + ay, ny);
                const long long n = ((long long)za * ny + y) * nx + x;
                const uint32_t inf = info[n];
                const bool ring2 = ax == 0 || ax == S::AX - 1 || ay == 0 || ay == S::AY - 1;
                T d0 = 0, d1 = 0;
                if (site_class(inf) == CLS_FLUID && (!ring2 || (inf & 0x7fffeu))) {
                    const NbrOffsets o(P, x, y, za);
                    pull_sum(fin, (unsigned)n, o, d0, d1);
                }
                sm.drho[slot][0][s] = d0;
                sm.drho[slot][1][s] = d1;
                sm.info[slot][s] = inf;
            }
        }
        __syncthreads();
        // ---------------- stage B: plane zb = z0 - 3 + k ----------------
        if (k >= 2) {
            const int zb_raw = z0 - 3 + k;
            const int zb = wrapc(zb_raw, nz);
            const int sl_m = (zb_raw - 1 + 8) % S::RING, sl_0 = (zb_raw + 8) % S::RING,
                      sl_p = (zb_raw + 1 + 8) % S::RING;
            for (int s = t; s < S::BN; s += S::NT) {
                const int bx = s % S::BX, by = s / S::BX;
                const int as = (by + 1) * S::AX + (bx + 1);
                const uint32_t cls = site_class(sm.info[sl_0][as]);
                T p0, p1;
                if (cls == CLS_FLUID) {
                    p0 = psi_dev(sm.drho[sl_0][0][as], e0, irho0);
                    p1 = psi_dev(sm.drho[sl_0][1][as], e1, irho0);
                } else if (cls == CLS_SHELL) {
                    T s0 = 0, s1 = 0;
                    int nf = 0;
#pragma unroll
                    for (int i = 1; i < Q; ++i) {
                        const int sl = cz(i) < 0 ? sl_m : (cz(i) > 0 ? sl_p : sl_0);
                        const int an = as + cy(i) * S::AX + cx(i);
                        if (site_class(sm.info[sl][an]) == CLS_FLUID) {
                            s0 += sm.drho[sl][0][an];
                            s1 += sm.drho[sl][1][an];
                            ++nf;
                        }
                    }
                    T r0 = nf ? s0 / (T)nf : (T)0, r1 = nf ? s1 / (T)nf : (T)0;
                    const int x = wrapc(x0 - 1 + bx, nx), y = wrapc(y0 - 1 + by, ny);
                    const double col = D.color[owner[((long long)zb * ny + y) * nx + x]];
                    if (col > 0.0) r0 += (T)fabs(col);
                    if (col < 0.0) r1 += (T)fabs(col);
                    sm.drho[sl_0][0][as] = r0;  // shell slot: read by stage C of this plane only
                    sm.drho[sl_0][1][as] = r1;
                    p0 = psi_dev(r0, e0, irho0);
                    p1 = psi_dev(r1, e1, irho0);
                } else {
                    p0 = psolid0;
                    p1 = psolid1;
                }
                sm.psi[sl_0][0][s] = p0;
                sm.psi[sl_0][1][s] = p1;
            }
        }
        __syncthreads();
        // ---------------- stage C: plane zc = z0 - 4 + k ----------------
        if (k >= 4 && mine) {
            const int zc = z0 - 4 + k;  // inside [z0, zend)
            const int sl_m = (zc - 1 + 8) % S::RING, sl_0 = (zc + 8) % S::RING, sl_p = (zc + 1 + 8) % S::RING;
            const int as = (ty + 2) * S::AX + (tx + 2);
            const int bs = (ty + 1) * S::BX + (tx + 1);
            const uint32_t inf = sm.info[sl_0][as];
            const uint32_t cls = site_class(inf);
            const long long n = ((long long)zc * ny + ys) * nx + xs;
            T f[2][Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) f[0][i] = f[1][i] = (T)0;  // the own slots of a non-fluid site
            if (cls == CLS_FLUID || cls == CLS_SHELL) {
                // Eq. (4) from the Psi ring
                T pn[2][Q - 1], acc[2][3];
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    const int sl = cz(i) < 0 ? sl_m : (cz(i) > 0 ? sl_p : sl_0);
                    const int bn = bs + cy(i) * S::BX + cx(i);
                    pn[0][i - 1] = sm.psi[sl][0][bn];
                    pn[1][i - 1] = sm.psi[sl][1][bn];
                }
                psi_force_sum(P, pn, acc);
                if (cls == CLS_SHELL) {
                    const T ps0 = psi_of(sm.drho[sl_0][0][as] + ref0, rho0, irho0);
                    const T ps1 = psi_of(sm.drho[sl_0][1][as] + ref1, rho0, irho0);
                    T F[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) F[a] = -ps0 * g * acc[1][a] - ps1 * g * acc[0][a];
                    if (shell_force_in_slots<T>(inf)) {
                        put_shell_force(f, F, inf);
                    } else {
#pragma unroll
                        for (int a = 0; a < 3; ++a) fsc[vidx(a, (unsigned)n)] = F[a];
                    }
                } else {
                    const NbrOffsets o(P, xs, ys, zc);
                    pull_load(fin, (unsigned)n, o, f);
                    collide_site<M>(P, f, acc, inf, (unsigned)n, rho, mass0, mass1);
                }
            }
            Unroll<Q>::run([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                store_pop(fout, pidx(0, i, (unsigned)n), f[0][i], f[1][i]);
            });
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
        for (int w = 0; w < S::NT / 64; ++w) {
            s0 += sm.red[2 * w];
            s1 += sm.red[2 * w + 1];
        }
        partial[2 * blockIdx.x] = s0;
        partial[2 * blockIdx.x + 1] = s1;
    }
}

// ---------------------------------------------------------------------------
template <typename T, int TX, int TY>
static void launch_fused_t(lb_handle *h, const void *fin, void *fout) {
    const int ntx = (h->prm.nx + TX - 1) / TX, nty = (h->prm.ny + TY - 1) / TY;
    const int TZ = h->fused_tz;
    const int nseg = (h->prm.nz + TZ - 1) / TZ;
    const unsigned nb = (unsigned)(ntx * nty * nseg);
    with_model(h->prm, [&](auto m) {
        k_fused_step<T, TX, TY, decltype(m)><<<nb, TX * TY, 0, h->stream>>>(
            h->dp, h->dpart, (const T *)fin, (T *)fout, (T *)h->rho, h->info, h->owner, (T *)h->fsc, h->partial, TZ,
            ntx, nty);
    });
    LB_HIP_CHECK(hipGetLastError());
    h->n_fused_blocks = (int)nb;
}

// the halo coordinates stay within one period of the box when the tile is at
// most the box edge minus 2 (x, y) and the z segment shorter than the box
bool fused_supported(const lb_params &p) { return p.nx >= 18 && p.ny >= 10 && p.nz >= 4; }

void launch_fused(lb_handle *h, const void *fin, void *fout) {
    const int tx = h->fused_tx, ty = h->fused_ty;
    if (h->prm.precision == LB_FP64) {
        if (tx == 32 && ty == 4) launch_fused_t<double, 32, 4>(h, fin, fout);
        else launch_fused_t<double, 16, 8>(h, fin, fout);
    } else {
        if (tx == 64 && ty == 4) launch_fused_t<float, 64, 4>(h, fin, fout);
        else if (tx == 32 && ty == 8) launch_fused_t<float, 32, 8>(h, fin, fout);
        else if (tx == 32 && ty == 4) launch_fused_t<float, 32, 4>(h, fin, fout);
        else launch_fused_t<float, 16, 8>(h, fin, fout);
    }
}

}  // namespace lbm
