// Device-side building blocks of the gfx950 lattice Boltzmann library: the
// D3Q19 lattice, the per-handle parameter block passed to every kernel, the
// equilibrium of Eq. (3), the effective mass of Eq. (5), the exact fixed-point
// inside test of the sphere discretisation (Sec. III) and deterministic
// block reductions (fixed order, no floating-point atomics).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 19;
constexpr int BLOCK = 256;  // threads per block of the generic kernels (4 wave64)

// D3Q19 velocities in the order of the public layout (rest, 6 faces, 12 edges,
// opposite directions adjacent).
__host__ __device__ constexpr int cx(int i) {
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
         : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
}
__host__ __device__ constexpr int cy(int i) {
    return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
         : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
}
__host__ __device__ constexpr int cz(int i) {
    return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
         : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr int norm2(int i) { return cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i); }
// lattice weights zeta_i (standard D3Q19: 1/3, 1/18, 1/36)
__host__ __device__ constexpr double zeta(int i) {
    return norm2(i) == 0 ? 1.0 / 3.0 : (norm2(i) == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// per-site classification word: bits 1..18 flag the directions i whose
// neighbour x + c_i is solid (bounce-back), bits 29..30 hold the class
enum : uint32_t { CLS_FLUID = 0, CLS_SHELL = 1, CLS_SOLID = 2, CLS_WALL = 3 };
constexpr int CLS_SHIFT = 29;
__host__ __device__ inline uint32_t site_class(uint32_t info) { return (info >> CLS_SHIFT) & 3u; }

constexpr int32_t OWN_FLUID = -1, OWN_WALL_LO = -2, OWN_WALL_HI = -3;
constexpr int32_t STAGE_NONE = 0x7fffffff;

struct DevParams {
    int nx, ny, nz, np;
    long long N;
    double tau[2];
    double g, rho0, w_face, w_edge;
    int velocity_mode, eq_order, wall_axis, pad;
    double rho_init[2];
    double rho_ref[2];  // populations are stored as f_i - zeta_i rho_ref^c
    double psi_e[2];    // rho0 exp(-rho_ref^c / rho0): Psi(rho_ref + d) - Psi(rho_ref) = -psi_e expm1(-d/rho0)
    double body[3];
    double wall_vel[2][3];
    double c0;
    double k_hertz, lub_hc, lub_hmin, nu;
};

// device-resident scalars of a handle
struct DevState {
    double M0[2];      // fluid mass at the start of the first step
    double Mstep[2];   // fluid mass at the start of the current step
    int32_t have_M0;
    int32_t unstable;
    int32_t overflow;  // bit 0 links, bit 1 shell, bit 2 events, bit 3 a sphere moved >= 1 site
    int32_t pad;
    unsigned long long covered_total, uncovered_total, refill_fallback;
};

// per-particle arrays (FP64), each np*3 unless noted
struct DevParticles {
    double *R, *U, *W, *Rprev;
    double *Ffl, *Tfl, *Ftot, *Ttot, *P, *PT;
    double *rad, *mass, *inertia, *color;  // np each
    int32_t *prescribed;
    // per-particle list segments (offset into the flat arrays, capacity, count)
    int32_t *link_off, *link_cap, *link_cnt;
    int64_t *links;  // site * 32 + direction (push view: site + c_dir is solid)
    int32_t *shell_off, *shell_cap, *shell_cnt;
    int32_t *shell;
    int32_t *ev_off, *ev_cap, *cov_cnt, *unc_cnt;
    int32_t *cov, *unc;
};

__device__ __forceinline__ int wrapc(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }
__device__ __forceinline__ int wrapany(int a, int n) { a %= n; return a < 0 ? a + n : a; }

// equilibrium of Eq. (3) with c_s^2 = 1/3 for one direction
template <typename C>
__device__ __forceinline__ C feq_dir(int i, C rho, C ux, C uy, C uz, C u2, int order) {
    const C cu = C(cx(i)) * ux + C(cy(i)) * uy + C(cz(i)) * uz;
    C b = C(1) + C(3) * cu + C(4.5) * cu * cu - C(1.5) * u2;
    if (order >= 3) b += C(4.5) * cu * cu * cu - C(4.5) * u2 * cu;
    return C(zeta(i)) * rho * b;
}

// f^eq_i - zeta_i rho_ref = zeta_i [ (rho - rho_ref) + rho (bracket - 1) ]: the
// equilibrium as a deviation from the stored reference, all terms small
template <typename C>
__device__ __forceinline__ C feq_dev_dir(int i, C drho, C rho, C ux, C uy, C uz, C u2, int order) {
    const C cu = C(cx(i)) * ux + C(cy(i)) * uy + C(cz(i)) * uz;
    C b = C(3) * cu + C(4.5) * cu * cu - C(1.5) * u2;
    if (order >= 3) b += C(4.5) * cu * cu * cu - C(4.5) * u2 * cu;
    return C(zeta(i)) * (drho + rho * b);
}

template <typename C>
__device__ __forceinline__ C psi_of(C rho, C rho0) { return rho0 * (C(1) - exp(-rho / rho0)); }

// Psi(rho_ref + d) - Psi(rho_ref) from the density deviation d; the neighbour
// sum of Eq. (4) only sees differences of Psi because sum_i W_i c_i = 0
template <typename C>
__device__ __forceinline__ C psi_dev(C d, C e, C rho0) { return -e * expm1(-d / rho0); }

// ---------------------------------------------------------------------------
// Sphere discretisation: site inside iff |x - R|^2 < r^2, evaluated on the
// centre and radius rounded to multiples of 2^-20 in 64-bit integers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long fixed20(double v) { return __double2ll_rn(v * 1048576.0); }

__device__ __forceinline__ bool inside_sphere(int x, int y, int z, const long long cq[3], long long r2q,
                                              int nx, int ny, int nz) {
    const int pos[3] = {x, y, z};
    const int L[3] = {nx, ny, nz};
    long long d2 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long Lq = (long long)L[a] << 20;
        long long d = (((long long)pos[a] << 20) - cq[a]) % Lq;  // in (-Lq, Lq)
        if (d > Lq / 2) d -= Lq;
        else if (d <= -(Lq / 2)) d += Lq;
        d2 += d * d;
    }
    return d2 < r2q;
}

// inclusive integer bounding box that contains every site inside the sphere;
// empty (hi < lo) for a centre that is not finite or far outside the box
__device__ __forceinline__ void sphere_box(const double R[3], double r, int lo[3], int hi[3]) {
    bool ok = isfinite(r) && r >= 0.0 && r < 1.0e4;
#pragma unroll
    for (int a = 0; a < 3; ++a) ok = ok && isfinite(R[a]) && fabs(R[a]) < 1.0e6;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = ok ? (int)floor(R[a] - r) - 1 : 0;
        hi[a] = ok ? (int)ceil(R[a] + r) + 1 : -1;
    }
}

// minimum-image displacement for |d| < L (one wrap; no loop, so a
// non-finite value passes through instead of spinning)
__device__ __forceinline__ double minimg(double d, double L) {
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

__device__ __forceinline__ void site_xyz(long long n, const DevParams &P, int &x, int &y, int &z) {
    const long long nxy = (long long)P.nx * P.ny;
    z = (int)(n / nxy);
    const int r = (int)(n - (long long)z * nxy);
    y = r / P.nx;
    x = r - y * P.nx;
}

__device__ __forceinline__ long long site_of(int x, int y, int z, const DevParams &P) {
    return ((long long)z * P.ny + y) * P.nx + x;
}

// the site's class word from the owner map: bounce-back directions of a
// fluid site, or shell / interior / wall for the others
__device__ __forceinline__ uint32_t compute_info(long long n, const DevParams &P, const int32_t *__restrict__ owner) {
    int x, y, z;
    site_xyz(n, P, x, y, z);
    const int32_t own = owner[n];
    if (own == OWN_WALL_LO || own == OWN_WALL_HI) return (uint32_t)CLS_WALL << CLS_SHIFT;
    uint32_t mask = 0;
    bool any_fluid = false;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const long long m = site_of(wrapc(x + cx(i), P.nx), wrapc(y + cy(i), P.ny), wrapc(z + cz(i), P.nz), P);
        const int32_t o = owner[m];
        if (o != OWN_FLUID) mask |= 1u << i;
        else any_fluid = true;
    }
    if (own == OWN_FLUID) return mask;
    return (uint32_t)(any_fluid ? CLS_SHELL : CLS_SOLID) << CLS_SHIFT;
}

// velocity of the solid at the midpoint of the link from fluid site x along
// c_i into the solid site x + c_i (owner own: particle or wall)
__device__ __forceinline__ void solid_velocity(const DevParams &P, const DevParticles &D, int32_t own, int x, int y,
                                               int z, int i, double ub[3], double rb[3]) {
    if (own >= 0) {
        const double mid[3] = {x + 0.5 * cx(i), y + 0.5 * cy(i), z + 0.5 * cz(i)};
        const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
#pragma unroll
        for (int a = 0; a < 3; ++a) rb[a] = minimg(mid[a] - D.R[3 * own + a], L[a]);
        const double *U = &D.U[3 * own], *W = &D.W[3 * own];
        ub[0] = U[0] + (W[1] * rb[2] - W[2] * rb[1]);
        ub[1] = U[1] + (W[2] * rb[0] - W[0] * rb[2]);
        ub[2] = U[2] + (W[0] * rb[1] - W[1] * rb[0]);
    } else {
        const int wi = own == OWN_WALL_LO ? 0 : 1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ub[a] = P.wall_vel[wi][a];
            rb[a] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// deterministic block reductions (blockDim.x == BLOCK)
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double *lds /* K*BLOCK */) {
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < K; ++k) lds[k * BLOCK + t] = v[k];
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int k = 0; k < K; ++k) lds[k * BLOCK + t] += lds[k * BLOCK + t + s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = lds[k * BLOCK];
    __syncthreads();
}

// Order-preserving compaction of one flag per thread: returns the slot of a
// flagged thread (base + number of flagged threads with smaller index) and
// advances base by the block total.  lds: at least BLOCK/64 + 1 ints.
__device__ __forceinline__ int block_compact(bool flag, int &base, int *lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long ballot = __ballot(flag);
    const int in_wave = __popcll(ballot & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    if (lane == 0) lds[wave] = __popcll(ballot);
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < BLOCK / 64; ++w) {
        const int c = lds[w];
        if (w < wave) before += c;
        total += c;
    }
    __syncthreads();
    const int slot = base + before + in_wave;
    base += total;
    return slot;
}

}  // namespace lbm
