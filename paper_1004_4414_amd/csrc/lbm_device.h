// Device-side building blocks of the gfx950 lattice Boltzmann library: the
// D3Q19 lattice, the per-handle parameter block passed to every kernel, the
// equilibrium of Eq. (3), the effective mass of Eq. (5), the exact fixed-point
// inside test of the sphere discretisation (Sec. III) and deterministic
// block reductions (fixed order, no floating-point atomics).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <type_traits>

namespace lbm {

// compile-time loop: f(integral_constant<int, 0>) ... f(integral_constant<int, I-1>),
// so that arrays indexed by the loop variable stay in registers
template <int I>
struct Unroll {
    template <class F>
    __device__ __forceinline__ static void run(F &&f) {
        Unroll<I - 1>::run(f);
        f(std::integral_constant<int, I - 1>{});
    }
};
template <>
struct Unroll<0> {
    template <class F>
    __device__ __forceinline__ static void run(F &&) {}
};

constexpr int Q = 19;
constexpr int BLOCK = 256;  // threads per block of the generic kernels (4 wave64)

// D3Q19 velocities in the order of the public layout (rest, 6 faces, 12 edges,
// opposite directions adjacent).
// (each component as two bit sets over the direction index, so that a
// runtime direction costs two shifts and no branches)
constexpr uint32_t DIRSET_PX = (1u << 1) | (1u << 7) | (1u << 9) | (1u << 11) | (1u << 13);
constexpr uint32_t DIRSET_MX = (1u << 2) | (1u << 8) | (1u << 10) | (1u << 12) | (1u << 14);
constexpr uint32_t DIRSET_PY = (1u << 3) | (1u << 7) | (1u << 10) | (1u << 15) | (1u << 17);
constexpr uint32_t DIRSET_MY = (1u << 4) | (1u << 8) | (1u << 9) | (1u << 16) | (1u << 18);
constexpr uint32_t DIRSET_PZ = (1u << 5) | (1u << 11) | (1u << 14) | (1u << 15) | (1u << 18);
constexpr uint32_t DIRSET_MZ = (1u << 6) | (1u << 12) | (1u << 13) | (1u << 16) | (1u << 17);
__host__ __device__ constexpr int cx(int i) { return (int)((DIRSET_PX >> i) & 1u) - (int)((DIRSET_MX >> i) & 1u); }
__host__ __device__ constexpr int cy(int i) { return (int)((DIRSET_PY >> i) & 1u) - (int)((DIRSET_MY >> i) & 1u); }
__host__ __device__ constexpr int cz(int i) { return (int)((DIRSET_PZ >> i) & 1u) - (int)((DIRSET_MZ >> i) & 1u); }
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr int norm2(int i) { return i == 0 ? 0 : (i <= 6 ? 1 : 2); }
// lattice weights zeta_i (standard D3Q19: 1/3, 1/18, 1/36)
__host__ __device__ constexpr double zeta(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }
static_assert(cx(7) == 1 && cy(7) == 1 && cz(7) == 0 && cx(18) == 0 && cy(18) == -1 && cz(18) == 1, "D3Q19 table");
static_assert(cx(opp(13)) == -cx(13) && cz(opp(13)) == -cz(13) && norm2(12) == 2 && norm2(6) == 1, "D3Q19 table");

// ---------------------------------------------------------------------------
// Memory layout.  Sites are grouped in storage blocks of VB = 64 consecutive
// linear indices (one wavefront).  A block keeps all its populations
// together, one run of 64 sites per direction, the two components of a site
// side by side: population (c, i) of site n lives at
//   (n / 64) * (2*19*64) + i * 128 + 2 * (n % 64) + c,
// so a wavefront's load of one direction (both components) is a single
// aligned 512-byte run, and one bounce-back link touches one 8-byte pair.
// The whole block spans a few pages (a plane-per-direction layout would make
// every wavefront touch ~80 pages and thrash the L1 TLB).  Two-component
// fields are stored as pairs per site, 3-vectors padded to four.
// ---------------------------------------------------------------------------
constexpr unsigned VB = 64;
__host__ __device__ __forceinline__ size_t pidx(int c, int i, unsigned n) {
    return (size_t)(n / VB) * (2 * Q * VB) + (size_t)i * (2 * VB) + 2 * (size_t)(n % VB) + c;
}
__host__ __device__ __forceinline__ size_t sidx(int c, unsigned n) { return 2 * (size_t)n + c; }
__host__ __device__ __forceinline__ size_t vidx(int a, unsigned n) { return 4 * (size_t)n + a; }

// component pairs as one vector access
template <typename T>
struct PairOf;
template <>
struct PairOf<float> {
    using type = float2;
};
template <>
struct PairOf<double> {
    using type = double2;
};
template <typename T>
using Pair = typename PairOf<T>::type;
// the pair at element index k (even) of an array of the arithmetic type
template <typename T>
__device__ __forceinline__ Pair<T> load_pair(const T *__restrict__ a, size_t k) {
    return *reinterpret_cast<const Pair<T> *>(a + k);
}
template <typename T>
__device__ __forceinline__ void store_pair(T *__restrict__ a, size_t k, T v0, T v1) {
    Pair<T> v;
    v.x = v0;
    v.y = v1;
    *reinterpret_cast<Pair<T> *>(a + k) = v;
}

// Population storage types.  S is the stored scalar and Cmp<S> the type the
// arithmetic runs in: FP64 and FP32 store what they compute; FP16 and BF16
// store the deviations f_i - zeta_i rho_ref rounded to nearest, and every
// update runs in FP32.  Populations move as component pairs (4, 8 or 16 B).
//
// A population written in one step is read back only in the next one, long
// after the caches have turned over, so every population store carries the
// non-temporal hint: it does not displace the lines that the sweep still
// reads (the x-shifted pulls and the Psi neighbours).  load_stream is the
// same hint on a load whose lines no other wavefront of the sweep reads;
// store_keep is a store with the default policy, for the scattered 8-byte
// bounce-back writes of the sphere links, whose partly written lines are
// better left in the caches until the next sweep reads them (wall links
// fill whole planes and keep the hint).
typedef float NtF2 __attribute__((ext_vector_type(2)));
typedef double NtD2 __attribute__((ext_vector_type(2)));
template <typename V, typename P>
__device__ __forceinline__ void nt_store(P *at, V v) {
    __builtin_nontemporal_store(v, reinterpret_cast<V *>(at));
}
// a component pair of a field in the arithmetic type, with the same hint
template <typename T>
__device__ __forceinline__ void store_pair_stream(T *__restrict__ a, size_t k, T v0, T v1) {
    typedef T V __attribute__((ext_vector_type(2)));
    nt_store(a + k, V{v0, v1});
}
// two 16-bit values as one 32-bit word, x in the low half (the order of the
// pair types); composed with shifts because a bit copy of the pair type can
// lose the non-temporal hint of the store that follows
__device__ __forceinline__ uint32_t pack16(uint32_t lo, uint32_t hi) { return lo | (hi << 16); }
template <typename S>
struct Storage;
template <>
struct Storage<double> {
    using T = double;
    __device__ static double2 load(const double *a, size_t k) { return *reinterpret_cast<const double2 *>(a + k); }
    __device__ static double2 load_stream(const double *a, size_t k) {
        const NtD2 v = __builtin_nontemporal_load(reinterpret_cast<const NtD2 *>(a + k));
        return make_double2(v.x, v.y);
    }
    __device__ static double rt(double x) { return x; }
    __device__ static void store(double *a, size_t k, double x, double y) { nt_store(a + k, NtD2{x, y}); }
    __device__ static void store_keep(double *a, size_t k, double x, double y) {
        *reinterpret_cast<double2 *>(a + k) = make_double2(x, y);
    }
};
template <>
struct Storage<float> {
    using T = float;
    __device__ static float2 load(const float *a, size_t k) { return *reinterpret_cast<const float2 *>(a + k); }
    __device__ static float2 load_stream(const float *a, size_t k) {
        const NtF2 v = __builtin_nontemporal_load(reinterpret_cast<const NtF2 *>(a + k));
        return make_float2(v.x, v.y);
    }
    __device__ static float rt(float x) { return x; }
    __device__ static void store(float *a, size_t k, float x, float y) { nt_store(a + k, NtF2{x, y}); }
    __device__ static void store_keep(float *a, size_t k, float x, float y) {
        *reinterpret_cast<float2 *>(a + k) = make_float2(x, y);
    }
};
template <>
struct Storage<__half> {
    using T = float;
    __device__ static float2 load(const __half *a, size_t k) {
        return __half22float2(*reinterpret_cast<const __half2 *>(a + k));
    }
    __device__ static float2 load_stream(const __half *a, size_t k) {
        const uint32_t u = __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(a + k));
        return make_float2(__half2float(__ushort_as_half((unsigned short)(u & 0xffffu))),
                           __half2float(__ushort_as_half((unsigned short)(u >> 16))));
    }
    __device__ static void store(__half *a, size_t k, float x, float y) {
        nt_store(a + k, pack16(__half_as_ushort(__float2half_rn(x)), __half_as_ushort(__float2half_rn(y))));
    }
    // the value a store_keep followed by a load gives back
    __device__ static float rt(float x) { return __half22float2(__floats2half2_rn(x, x)).x; }
    __device__ static void store_keep(__half *a, size_t k, float x, float y) {
        *reinterpret_cast<__half2 *>(a + k) = __floats2half2_rn(x, y);
    }
};
template <>
struct Storage<__hip_bfloat16> {
    using T = float;
    __device__ static float2 load(const __hip_bfloat16 *a, size_t k) {
        return __bfloat1622float2(*reinterpret_cast<const __hip_bfloat162 *>(a + k));
    }
    __device__ static float2 load_stream(const __hip_bfloat16 *a, size_t k) {
        const uint32_t u = __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(a + k));
        return make_float2(__bfloat162float(__ushort_as_bfloat16((unsigned short)(u & 0xffffu))),
                           __bfloat162float(__ushort_as_bfloat16((unsigned short)(u >> 16))));
    }
    __device__ static void store(__hip_bfloat16 *a, size_t k, float x, float y) {
        nt_store(a + k, pack16(__bfloat16_as_ushort(__float2bfloat16(x)), __bfloat16_as_ushort(__float2bfloat16(y))));
    }
    __device__ static float rt(float x) { return __bfloat1622float2(__float22bfloat162_rn(make_float2(x, x))).x; }
    __device__ static void store_keep(__hip_bfloat16 *a, size_t k, float x, float y) {
        *reinterpret_cast<__hip_bfloat162 *>(a + k) = __float22bfloat162_rn(make_float2(x, y));
    }
};
template <typename S>
using Cmp = typename Storage<S>::T;
template <typename S>
__device__ __forceinline__ Pair<Cmp<S>> load_pop(const S *__restrict__ a, size_t k) {
    return Storage<S>::load(a, k);
}
template <typename S>
__device__ __forceinline__ void store_pop(S *__restrict__ a, size_t k, Cmp<S> v0, Cmp<S> v1) {
    Storage<S>::store(a, k, v0, v1);
}
template <typename S>
__device__ __forceinline__ void store_pop_keep(S *__restrict__ a, size_t k, Cmp<S> v0, Cmp<S> v1) {
    Storage<S>::store_keep(a, k, v0, v1);
}
__host__ __device__ __forceinline__ size_t padded_sites(long long N) { return (size_t)((N + VB - 1) / VB) * VB; }

// division of 32-bit unsigned integers by an invariant divisor d via a
// multiply-high (Granlund & Montgomery 1994, round-up method):
// n / d = (t + ((n - t) >> s1)) >> s2 with t = mulhi(n, m)
struct FastDiv {
    uint32_t d, m;
    int s1, s2;
};
inline FastDiv make_fastdiv(uint32_t d) {
    int l = 0;
    while ((1ull << l) < d) ++l;
    FastDiv f;
    f.d = d;
    f.m = (uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
    f.s1 = l < 1 ? l : 1;
    f.s2 = l > 1 ? l - 1 : 0;
    return f;
}
__device__ __forceinline__ uint32_t fast_div(uint32_t n, const FastDiv &f) {
    const uint32_t t = __umulhi(n, f.m);
    return (t + ((n - t) >> f.s1)) >> f.s2;
}

// per-site classification word: bits 1..18 flag the directions i whose
// neighbour x + c_i is solid (on fluid sites: the bounce-back links; on
// virtual-fluid sites: the complement of the fluid neighbours), bits 29..30
// hold the class
enum : uint32_t { CLS_FLUID = 0, CLS_SHELL = 1, CLS_SOLID = 2, CLS_WALL = 3 };
// bit 0 of a class word: the word was recomputed by the last map update (its
// site or a neighbour changed owner); no direction uses bit 0
constexpr uint32_t INFO_FLAG = 1u;
// bit 19 of a fluid site's class word: its solid neighbours belong to more
// than one sphere
constexpr uint32_t INFO_MULTI = 1u << 19;
constexpr int CLS_SHIFT = 29;
__host__ __device__ inline uint32_t site_class(uint32_t info) { return (info >> CLS_SHIFT) & 3u; }

constexpr int32_t OWN_FLUID = -1, OWN_WALL_LO = -2, OWN_WALL_HI = -3;
// stage[]: STAGE_NONE, or the new owner of a site whose owner changes in this
// step's map update (STAGE_FLUID for the fluid); the full rebuild instead
// takes the lowest index of the spheres that contain the site
constexpr int32_t STAGE_NONE = 0x7fffffff, STAGE_FLUID = 0x7ffffffe;

struct DevParams {
    int nx, ny, nz, np;
    long long N;
    double tau[2];
    double g, rho0, w_face, w_edge;
    int velocity_mode, eq_order, wall_axis, lub_mode;
    int any_color;  // any sphere with a non-zero colour (Sec. IV)
    // bounce-back of sphere links (set per launch): link_write = the link
    // kernel writes every bounced population into the solid site's slot;
    // otherwise redirect = this sweep forms them itself (sweep_bounce);
    // multi_bits: class words carry INFO_MULTI (lattices using that option)
    int link_write, redirect, multi_bits;
    int force_avg;  // the fluid force entering the leap-frog is averaged over two steps
    double rho_init[2];
    double rho_ref[2];  // populations are stored as f_i - zeta_i rho_ref^c
    double psi_e[2];    // rho0 exp(-rho_ref^c / rho0): Psi(rho_ref + d) - Psi(rho_ref) = -psi_e expm1(-d/rho0)
    double inv_tau[2];  // 1 / tau^c
    double inv_rho0;    // 1 / rho0
    FastDiv div_nx, div_nxy;
    double body[3];
    double wall_vel[2][3];
    double c0;
    double k_hertz, lub_hc, lub_hmin, nu;
};

// device-resident scalars of a handle
constexpr int FIN_BLOCKS = 256;   // most blocks of the fixed-order mass reduction
constexpr int FIN_PER_BLOCK = 1024;  // per-wavefront partial masses summed by one of them
// blocks of the mass reduction over nb partials
__host__ __device__ inline int fin_blocks(int nb) {
    const int n = (nb + FIN_PER_BLOCK - 1) / FIN_PER_BLOCK;
    return n < 1 ? 1 : (n > FIN_BLOCKS ? FIN_BLOCKS : n);
}
struct DevState {
    double M0[2];      // fluid mass at the start of the first step
    double Mstep[2];   // fluid mass at the start of the current step
    int32_t have_M0;
    int32_t unstable;
    int32_t overflow;  // bit 1 shell list, bit 2 event lists, bit 3 a sphere moved >= 1 site, bit 4 contacts
    int32_t pad;
    unsigned long long covered_total, uncovered_total, refill_fallback;
    double fin_part[2 * FIN_BLOCKS];  // per-block masses of the reduction (scratch)
    uint32_t fin_count;               // blocks done; back to 0 after every reduction
    uint32_t pad2;
};

// per-particle arrays (FP64), each np*3 unless noted
struct DevParticles {
    // Rprev: the centre at the last map update (the positions the solid map
    // holds)
    double *R, *U, *W, *Rprev;
    // candidate sites: Rscan is the centre of the last scan of the sphere's
    // box; cand lists the sites closer than margin (tau) to the surface of
    // the sphere centred there (bit 31 set on those inside) and ncand their
    // number.  While the fixed-point centre stays closer than tau to Rscan,
    // only those sites can change side, so a map update tests them alone.
    double *Rscan, *margin;
    int32_t *cand, *ncand;
    // the spheres whose centres were closer than r_a + r_b + NB_REACH at the
    // start of the step (the only ones that can share a site with this
    // sphere's old or new sites after a move of less than one site per axis);
    // nnbr > NB_CAP: too many to list, every sphere is tested instead
    int32_t *nbr, *nnbr;
    double *Ffl, *Tfl, *Ftot, *Ttot, *P, *PT;
    // np x 6: the fluid force and torque of the previous step (NaN: none yet)
    double *Fprev;
    double *rad, *mass, *inertia, *color;  // np each
    int32_t *prescribed;
    // per-particle list segments (offset into the flat arrays, capacity, count);
    // the bounce-back links of a sphere are those of its virtual-fluid sites
    // (a link (x, i) ends on the solid site x + c_i, which has the fluid
    // neighbour x), so only their number is kept
    int32_t *link_cnt;
    int32_t *shell_off, *shell_cap, *shell_cnt;
    int32_t *shell;
    int32_t *ev_off, *ev_cap, *cov_cnt, *unc_cnt;
    int32_t *cov, *unc;
    // map-update bookkeeping: chg lists the sites whose owner changes this
    // step, found by sphere p (offset 2 ev_off, capacity 2 ev_cap; a site may
    // be listed by two spheres); dirty[] = coarse cells (CELL^3 sites) whose
    // class words changed
    int32_t *chg_cnt, *chg;
    int32_t *dirty;
    // running covered, uncovered and refill-fallback counts per sphere (np x 3)
    unsigned long long *evtot;
    // the previous step's change lists (for clearing its class-word flags);
    // track_flags: they are valid and the flags are cleared through them
    int32_t *chg_prev_cnt, *chg_prev;
    int track_flags;
    // the sphere state the link kernel used (np x 3 each): the moving-wall
    // term of a bounce formed later uses the same velocities and centre
    double *Rl, *Ul, *Wl;
    int32_t *lbox;  // np x 6: box (lo, ext) of the last list build
    // lubrication contacts (index order) and the velocities after every other force
    int32_t *ncont, *cont;    // np, np x MAX_LUB_CONTACTS
    double *cont_c, *cont_n;  // coefficient c and unit vector (lower to higher index) of each contact
    double *vs;               // np x 3
    int cgx, cgy, cgz;
    // cell list of the pair search (cells at least the interaction reach wide,
    // >= 3 per axis; pgx == 0: all pairs): counts (zero between steps), starts,
    // sphere indices grouped by cell, and the cell of each sphere
    int32_t *pc_cnt, *pc_start, *pc_items, *pc_of;
    int pgx, pgy, pgz;
};
constexpr int CELL_SHIFT = 3;  // coarse cells of 8^3 sites
constexpr int MAX_LUB_CONTACTS = 32;
constexpr int CAND_CAP = 256;  // near-surface sites kept per sphere
constexpr int NB_CAP = 32;     // listed neighbours per sphere
// neighbour reach beyond r_a + r_b: two moves of less than one site per axis
// (2 sqrt(3)) and the 2^-21 of the fixed-point radii
constexpr double NB_REACH = 3.5;


__device__ __forceinline__ int wrapc(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// The block a kernel body runs as and the number of blocks of its lattice:
// blockIdx.x / gridDim.x for a launch over one lattice, or a block's range
// within its member for a launch over a batch of lattices.
struct Grid {
    unsigned bid, nb;
};
__device__ __forceinline__ Grid own_grid() { return Grid{blockIdx.x, gridDim.x}; }

__device__ __forceinline__ bool dense_site(const DevParams &P, const Grid &g, unsigned &n, int &x, int &y, int &z) {
    const unsigned nb = g.nb;
    unsigned b = g.bid;
    if (nb % 8u == 0) b = (b % 8u) * (nb / 8u) + b / 8u;
    n = b * 256u + threadIdx.x;
    if (n >= (unsigned)P.N) return false;
    const unsigned zq = fast_div(n, P.div_nxy);
    const unsigned r = n - zq * P.div_nxy.d;
    const unsigned yq = fast_div(r, P.div_nx);
    x = (int)(r - yq * P.div_nx.d);
    y = (int)yq;
    z = (int)zq;
    return true;
}
// dense_site for boxes whose nx is a multiple of 64: a wavefront's 64 sites
// then lie in one row, so y and z are computed once per wavefront (scalar
// registers) from its first site; x = x0 + lane.
__device__ __forceinline__ bool dense_site(const DevParams &P, unsigned &n, int &x, int &y, int &z) {
    return dense_site(P, own_grid(), n, x, y, z);
}
__device__ __forceinline__ bool dense_site_rows(const DevParams &P, const Grid &g, unsigned &n, int &x, int &y,
                                                int &z) {
    const unsigned nb = g.nb;
    unsigned b = g.bid;
    if (nb % 8u == 0) b = (b % 8u) * (nb / 8u) + b / 8u;
    n = b * 256u + threadIdx.x;
    if (n >= (unsigned)P.N) return false;
    const unsigned n0 = __builtin_amdgcn_readfirstlane(n & ~63u);
    const unsigned zq = fast_div(n0, P.div_nxy);
    const unsigned r = n0 - zq * P.div_nxy.d;
    const unsigned yq = fast_div(r, P.div_nx);
    x = (int)(r - yq * P.div_nx.d + (n & 63u));
    y = (int)yq;
    z = (int)zq;
    return true;
}
// One lattice of a batch advanced by shared launches (one launch per stage of
// the step for all members): its parameters, sphere data and buffers for one
// step parity (fin / fout swap between the two tables of a batch).
struct BatchMember {
    DevParams P;
    DevParticles D;
    const void *fin;
    void *fout;
    void *rho, *psi, *fsc;
    uint32_t *info;
    int32_t *owner, *stage;
    double *partial;
    DevState *dstate;
    int rows;   // nx a multiple of 64: row-aligned addressing
    int cells;  // pair search by cell list
};
// Blocks of each member in a batched launch, as cumulative counts (nm + 1
// entries; a member with none has an empty range).
enum BatchMap : int {
    BM_DENSE = 0,    // blocks of the dense site grid
    BM_SPHERE,       // one block per sphere
    BM_SPHERE256,    // ceil(np / 256) blocks
    BM_CELL_SPHERE,  // one block per sphere, members with a cell list
    BM_CELL_SPH256,  // ceil(np / 256) blocks, members with a cell list
    BM_CELL_ONE,     // one block, members with a cell list
    BM_PAIR_SPHERE,  // one block per sphere, members with the all-pairs search
    BM_COUNT
};
struct BatchPlan {
    const BatchMember *m;
    const int32_t *start;  // BM_COUNT x (nm + 1)
    int nm;
};
// the member whose block range holds block b of a batched launch, and the
// block's place in it (uniform over the block)
__device__ __forceinline__ int batch_member(const BatchPlan &B, int map, Grid &g) {
    const int32_t *st = B.start + map * (B.nm + 1);
    const unsigned b = blockIdx.x;
    int lo = 0, hi = B.nm - 1;
    while (lo < hi) {  // last member whose start is <= b
        const int mid = (lo + hi + 1) >> 1;
        if ((unsigned)st[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const int m = __builtin_amdgcn_readfirstlane(lo);
    g.bid = b - (unsigned)st[m];
    g.nb = (unsigned)(st[m + 1] - st[m]);
    return m;
}

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

// exp(x) - 1 in FP32: Taylor polynomial to x^6 for |x| < 1/4 (truncation
// below 1.3e-8 relative), the hardware exponential elsewhere
__device__ __forceinline__ float fast_expm1(float x) {
    if (fabsf(x) < 0.25f)
        return x * (1.0f + x * (0.5f + x * (1.0f / 6 + x * (1.0f / 24 + x * (1.0f / 120 + x * (1.0f / 720))))));
    return __expf(x) - 1.0f;
}

// Eq. (5): Psi = rho0 (1 - exp(-rho/rho0)); FP32 uses the hardware exponential
__device__ __forceinline__ float psi_of(float rho, float rho0, float irho0) { return rho0 * (1.0f - __expf(-rho * irho0)); }
__device__ __forceinline__ double psi_of(double rho, double rho0, double irho0) {
    return rho0 * (1.0 - exp(-rho * irho0));
}

// Psi(rho_ref + d) - Psi(rho_ref) from the density deviation d; the neighbour
// sum of Eq. (4) only sees differences of Psi because sum_i W_i c_i = 0
__device__ __forceinline__ float psi_dev(float d, float e, float irho0) { return -e * fast_expm1(-d * irho0); }
__device__ __forceinline__ double psi_dev(double d, double e, double irho0) { return -e * expm1(-d * irho0); }

// dense launch geometry: one thread per site in linear order (a wavefront is
// one storage block), block ids remapped so that each XCD (the hardware deals
// block b to XCD b % 8) walks a contiguous slab of the box
__device__ __forceinline__ bool dense_site(const struct DevParams &P, unsigned &n, int &x, int &y, int &z);

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

// squared fixed-point distance of site (x, y, z) from the centre cq (minimum
// image), the quantity the inside test compares with r^2
// (x in [0, L) and a centre rounded from [0, L): one wrap suffices)
__device__ __forceinline__ long long dist2_sphere(int x, int y, int z, const long long cq[3], int nx, int ny, int nz) {
    const int pos[3] = {x, y, z};
    const int L[3] = {nx, ny, nz};
    long long d2 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long Lq = (long long)L[a] << 20;
        long long d = ((long long)pos[a] << 20) - cq[a];
        if (d > Lq / 2) d -= Lq;
        else if (d <= -(Lq / 2)) d += Lq;
        d2 += d * d;
    }
    return d2;
}
__device__ __forceinline__ long long dist2_unwrapped(const int u[3], const long long cq[3]) {
    long long d2 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long d = ((long long)u[a] << 20) - cq[a];
        d2 += d * d;
    }
    return d2;
}

// The same test on unwrapped box coordinates u (u = x mod L): equal to
// inside_sphere when every coordinate of the box lies within half a period
// of the centre, which near_box checks once per box.
__device__ __forceinline__ bool inside_unwrapped(const int u[3], const long long cq[3], long long r2q) {
    long long d2 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long d = ((long long)u[a] << 20) - cq[a];
        d2 += d * d;
    }
    return d2 < r2q;
}
__device__ __forceinline__ bool near_box(const int lo[3], const int ext[3], const long long cq[3], const DevParams &P) {
    const int L[3] = {P.nx, P.ny, P.nz};
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long h = ((long long)L[a] << 20) / 2;
        ok = ok && (((long long)lo[a] << 20) - cq[a] > -h) && (((long long)(lo[a] + ext[a] - 1) << 20) - cq[a] <= h);
    }
    return ok;
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
    const unsigned u = (unsigned)n;
    const unsigned zq = fast_div(u, P.div_nxy);
    const unsigned r = u - zq * P.div_nxy.d;
    const unsigned yq = fast_div(r, P.div_nx);
    x = (int)(r - yq * P.div_nx.d);
    y = (int)yq;
    z = (int)zq;
}

__device__ __forceinline__ long long site_of(int x, int y, int z, const DevParams &P) {
    return (long long)(((unsigned)z * (unsigned)P.ny + (unsigned)y) * (unsigned)P.nx + (unsigned)x);  // < N < 2^32
}

// the site's class word from the owner map: bounce-back directions of a
// fluid site, or shell / interior / wall for the others; MULTI: with the
// INFO_MULTI bit
template <bool MULTI>
__device__ __forceinline__ uint32_t class_word_at(long long n, int x, int y, int z, const DevParams &P,
                                                  const int32_t *__restrict__ owner) {
    const int32_t own = owner[n];
    if (own == OWN_WALL_LO || own == OWN_WALL_HI) return (uint32_t)CLS_WALL << CLS_SHIFT;
    uint32_t mask = 0;
    bool any_fluid = false, multi = false;
    int32_t first = OWN_FLUID;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const long long m = site_of(wrapc(x + cx(i), P.nx), wrapc(y + cy(i), P.ny), wrapc(z + cz(i), P.nz), P);
        const int32_t o = owner[m];
        if (o != OWN_FLUID) {
            mask |= 1u << i;
            if constexpr (MULTI) {
                multi = multi || (first != OWN_FLUID && o != first);
                first = o;
            }
        } else {
            any_fluid = true;
        }
    }
    if (own == OWN_FLUID) return multi ? mask | INFO_MULTI : mask;
    return any_fluid ? ((uint32_t)CLS_SHELL << CLS_SHIFT) | mask : (uint32_t)CLS_SOLID << CLS_SHIFT;
}
__device__ __forceinline__ uint32_t compute_info_at(long long n, int x, int y, int z, const DevParams &P,
                                                    const int32_t *__restrict__ owner) {
    return P.multi_bits ? class_word_at<true>(n, x, y, z, P, owner) : class_word_at<false>(n, x, y, z, P, owner);
}
__device__ __forceinline__ uint32_t compute_info(long long n, const DevParams &P, const int32_t *__restrict__ owner) {
    int x, y, z;
    site_xyz(n, P, x, y, z);
    return compute_info_at(n, x, y, z, P, owner);
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
        const bool lo = own == OWN_WALL_LO;  // select, not a runtime index into the parameter block
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ub[a] = lo ? P.wall_vel[0][a] : P.wall_vel[1][a];
            rb[a] = 0.0;
        }
    }
}

// c_i . u for the link from fluid site (x, y, z) along c_i into a sphere with
// centre R, velocity U and angular velocity W: u is the rigid velocity at x,
// which has the same component along c_i as at the link midpoint x + c_i/2
// (c_i . (W x c_i) = 0), Eq. (16)
__device__ __forceinline__ void rigid_u(const DevParams &P, const double R[3], const double U[3], const double W[3],
                                        int x, int y, int z, double u[3]) {
    // no contraction: every kernel that forms a bounced pair rounds alike
#pragma clang fp contract(off)
    const double r[3] = {minimg(x - R[0], (double)P.nx), minimg(y - R[1], (double)P.ny),
                         minimg(z - R[2], (double)P.nz)};
    u[0] = U[0] + (W[1] * r[2] - W[2] * r[1]);
    u[1] = U[1] + (W[2] * r[0] - W[0] * r[2]);
    u[2] = U[2] + (W[0] * r[1] - W[1] * r[0]);
}
__device__ __forceinline__ double cu_dot(int i, const double u[3]) {
#pragma clang fp contract(off)
    return (double)cx(i) * u[0] + (double)cy(i) * u[1] + (double)cz(i) * u[2];
}
__device__ __forceinline__ double rigid_cu(const DevParams &P, const double R[3], const double U[3], const double W[3],
                                           int x, int y, int z, int i) {
    double u[3];
    rigid_u(P, R, U, W, x, y, z, u);
    return cu_dot(i, u);
}

// the bounced pair of a link, Eq. (16): f*_i(x) - w^c with w^c = 6 zeta_i
// rho^c(x) (c_i . u_b), in stored (deviation) form: the reference parts of
// directions i and opp(i) are equal.  dr: the density deviations of x.
template <typename T>
__device__ __forceinline__ void bounce_pair(const DevParams &P, double cub, int i, T raw0, T raw1, T dr0, T dr1,
                                            T &b0, T &b1, T &w0, T &w1) {
#pragma clang fp contract(off)
    const T wz = (T)(6.0 * zeta(i) * cub);
    w0 = wz * (dr0 + (T)P.rho_ref[0]);
    w1 = wz * (dr1 + (T)P.rho_ref[1]);
    b0 = raw0 - w0;
    b1 = raw1 - w1;
}

// moments of one component from its stored values d_i = f_i - zeta_i rho_ref:
// dr = sum_i d_i, rho = dr + rho_ref, and j summed over opposite pairs (the
// reference part cancels exactly)
template <typename T>
__device__ __forceinline__ void moments(const T (&f)[Q], T ref, T &dr, T &r, T &jx, T &jy, T &jz) {
    dr = 0;
    Unroll<Q>::run([&](auto ic) { dr += f[decltype(ic)::value]; });
    r = dr + ref;
    jx = jy = jz = 0;
    Unroll<Q / 2>::run([&](auto ic) {
        constexpr int i = 2 * decltype(ic)::value + 1;
        const T d = f[i] - f[i + 1];
        if (cx(i)) jx += cx(i) > 0 ? d : -d;
        if (cy(i)) jy += cy(i) > 0 ? d : -d;
        if (cz(i)) jz += cz(i) > 0 ? d : -d;
    });
}

// Compile-time choices of the collision: velocity_mode 0 = common Shan-Chen
// velocity, 1 = per-component velocity (Sec. II); eq_order 2 or 3 (Eq. (3)).
template <int VM, int EO>
struct Model {
    static constexpr int velocity_mode = VM;
    static constexpr int eq_order = EO;
};

// reciprocal: the hardware approximation (1 ulp) in FP32, exact division in FP64
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// equilibrium velocities of both components (Sec. II, Eq. (6))
template <typename T, int VM>
__device__ __forceinline__ void eq_velocity(const DevParams &P, const T r[2], const T j[2][3], const T F[2][3],
                                            T ueq[2][3]) {
    T ubar[3] = {0, 0, 0};
    if (VM == 0) {
        const T it0 = (T)P.inv_tau[0], it1 = (T)P.inv_tau[1];
        const T den = r[0] * it0 + r[1] * it1;
        if (den != (T)0) {
            const T iden = recip(den);
#pragma unroll
            for (int a = 0; a < 3; ++a) ubar[a] = (j[0][a] * it0 + j[1][a] * it1) * iden;
        }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const T tau = (T)P.tau[c];
        // zero density: the component is inert (no velocity, no shift)
        const T ir = r[c] != (T)0 ? recip(r[c]) : (T)0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const T base = VM == 1 ? j[c][a] * ir : ubar[a];
            ueq[c][a] = base + tau * F[c][a] * ir;
        }
    }
}

// BGK relaxation, Eqs. (2), (3), of one component's stored deviations
// d_i = f_i - zeta_i rho_ref toward f^eq_i - zeta_i rho_ref, with opposite
// directions taken together: for the pair (i, opp(i)) the bracket of Eq. (3)
// minus one splits into a part even in c_i.u, 4.5 (c.u)^2 - 1.5 u^2, and an
// odd part, c.u (3 + 4.5 (c.u)^2 - 4.5 u^2) (third order) or 3 c.u.
template <typename T, int EO>
__device__ __forceinline__ void relax(T (&f)[Q], T dr, T r, T ux, T uy, T uz, T om) {
    const T u2 = ux * ux + uy * uy + uz * uz;
    const T m15u2 = (T)-1.5 * u2;
    const T k3 = EO >= 3 ? (T)3 - (T)4.5 * u2 : (T)3;
    {
        const T feq = (T)(1.0 / 3.0) * (dr + r * m15u2);
        f[0] = f[0] + om * (feq - f[0]);
    }
    const T zdr_f = (T)(1.0 / 18.0) * dr, zr_f = (T)(1.0 / 18.0) * r;
    const T zdr_e = (T)(1.0 / 36.0) * dr, zr_e = (T)(1.0 / 36.0) * r;
    Unroll<Q / 2>::run([&](auto kc) {
        constexpr int i = 2 * decltype(kc)::value + 1;  // i + 1 = opp(i)
        T cu = 0;
        if (cx(i)) cu += cx(i) > 0 ? ux : -ux;
        if (cy(i)) cu += cy(i) > 0 ? uy : -uy;
        if (cz(i)) cu += cz(i) > 0 ? uz : -uz;
        const T cu2 = cu * cu;
        const T even = (T)4.5 * cu2 + m15u2;
        const T odd = EO >= 3 ? cu * ((T)4.5 * cu2 + k3) : (T)3 * cu;
        const T zr = norm2(i) == 1 ? zr_f : zr_e, zdr = norm2(i) == 1 ? zdr_f : zdr_e;
        const T A = zdr + zr * even, B = zr * odd;
        f[i] = f[i] + om * ((A + B) - f[i]);
        f[i + 1] = f[i + 1] + om * ((A - B) - f[i + 1]);
    });
}

// Eq. (4) neighbour sum: acc[c][a] = sum_{i=1..18} W_i pn[c][i-1] c_ia with
// pn = Psi^c(x + c_i) - Psi^c(rho_ref) (the constant drops out because
// sum_i W_i c_i = 0); faces and edges summed separately as opposite-pair
// differences, then weighted
template <typename T>
__device__ __forceinline__ void psi_force_sum(const DevParams &P, const T (&pn)[2][Q - 1], T (&acc)[2][3]) {
    const T wf = (T)P.w_face, we = (T)P.w_edge;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const T sf[3] = {pn[c][0] - pn[c][1], pn[c][2] - pn[c][3], pn[c][4] - pn[c][5]};
        T se[3] = {0, 0, 0};
        Unroll<6>::run([&](auto kc) {
            constexpr int i = 7 + 2 * decltype(kc)::value;  // edge pair (i, i + 1)
            const T d = pn[c][i - 1] - pn[c][i];
            if (cx(i)) se[0] += cx(i) > 0 ? d : -d;
            if (cy(i)) se[1] += cy(i) > 0 ? d : -d;
            if (cz(i)) se[2] += cz(i) > 0 ? d : -d;
        });
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[c][a] = wf * sf[a] + we * se[a];
    }
}

// ---------------------------------------------------------------------------
// Population storage (pull form).  Slot (c, i, z) of a buffer holds the value
// that site z + c_i receives in direction i: the post-streaming population of
// a fluid site x is f_i(x) = slot (i, x - c_i).  The sweep reads those slots,
// collides and writes the own slots (i, x) of every site, solid ones included
// (zeros), so that every store instruction covers whole 512-byte runs: stores
// with lanes masked off leave partly written lines that HBM writes back far
// more slowly.  When x + c_i is solid, f*_i(x) in slot (i, x) is read by the
// link kernels after the sweep, which write the bounced population (with the
// moving-wall term) into the solid site's slot (opp(i), x + c_i), exactly
// where x reads direction opp(i) at the next step.
// ---------------------------------------------------------------------------

// signed offsets from a site to its 18 neighbours with the periodic wrap folded
// into per-axis corrections (32-bit site indices)
struct NbrOffsets {
    int nx, nxy, xm, xp, ym, yp, zm, zp;
    __device__ __forceinline__ NbrOffsets(const DevParams &P, int xs, int ys, int zs) {
        nx = P.nx;
        nxy = P.nx * P.ny;
        const int N = (int)P.N;
        xm = xs == 0 ? nx : 0;
        xp = xs == P.nx - 1 ? -nx : 0;
        ym = ys == 0 ? nxy : 0;
        yp = ys == P.ny - 1 ? -nxy : 0;
        zm = zs == 0 ? N : 0;
        zp = zs == P.nz - 1 ? -N : 0;
    }
    template <int i>
    __device__ __forceinline__ int off() const {
        return cx(i) + cy(i) * nx + cz(i) * nxy + (cx(i) < 0 ? xm : (cx(i) > 0 ? xp : 0)) +
               (cy(i) < 0 ? ym : (cy(i) > 0 ? yp : 0)) + (cz(i) < 0 ? zm : (cz(i) > 0 ? zp : 0));
    }
};

// f_i(x) = slot (i, x - c_i) for both components
template <typename S, typename T = Cmp<S>>
__device__ __forceinline__ void pull_load(const S *__restrict__ fin, unsigned n, const NbrOffsets &o, T (&f)[2][Q]) {
    Unroll<Q>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const unsigned src = i == 0 ? n : (unsigned)((int)n + o.template off<opp(i)>());
        const Pair<T> v = load_pop(fin, pidx(0, i, src));
        f[0][i] = v.x;
        f[1][i] = v.y;
    });
}

// ---------------------------------------------------------------------------
// Row-aligned addressing (nx a multiple of 64, sites from dense_site_rows).
// Every row that a wavefront's pulls, Psi reads and own stores touch is the
// same for all of its lanes, so the row's byte offset is wavefront-uniform
// (scalar arithmetic) and a lane adds a 32-bit offset that depends only on
// its x and the direction's x step.  The addresses are those of pidx / sidx:
// with m = R nx + x (R the row), m / 64 = R nx/64 + x/64 and m % 64 = x % 64.
// ---------------------------------------------------------------------------
template <typename S>
struct RowView {
    using T = Cmp<S>;
    static constexpr uint32_t PB = 2 * sizeof(S);           // a component pair
    static constexpr uint32_t DB = 2 * VB * sizeof(S);      // one direction of a storage block
    static constexpr uint32_t BB = 2 * Q * VB * sizeof(S);  // a storage block
    static constexpr uint32_t FB = 2 * sizeof(T);           // a pair of a two-component field
    int ys[3], zs[3];  // y - 1, y, y + 1 and z - 1, z, z + 1, wrapped (wavefront-uniform)
    uint32_t po[3];    // byte offset within a row of the storage of x + dx, dx = -1, 0, 1
    uint32_t fo[3];    // byte offset within a row of a field pair of x + dx
    uint64_t prow, frow;
    int ny;
    __device__ __forceinline__ RowView(const DevParams &P, int x, int y, int z) {
        const int nx = P.nx;
        ny = P.ny;
        ys[1] = y;
        ys[0] = y == 0 ? P.ny - 1 : y - 1;
        ys[2] = y == P.ny - 1 ? 0 : y + 1;
        zs[1] = z;
        zs[0] = z == 0 ? P.nz - 1 : z - 1;
        zs[2] = z == P.nz - 1 ? 0 : z + 1;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            int xs = x + k - 1;
            xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
            po[k] = (uint32_t)(xs / (int)VB) * BB + (uint32_t)(xs % (int)VB) * PB;
            fo[k] = (uint32_t)xs * FB;
        }
        prow = (uint64_t)(nx / (int)VB) * BB;
        frow = (uint64_t)nx * FB;
    }
    __device__ __forceinline__ uint64_t row(int dy, int dz) const {
        return (uint64_t)(uint32_t)(zs[dz + 1] * ny + ys[dy + 1]);
    }
};

// One row-aligned pull of direction i by a wavefront.  With c_ix = 0 it reads
// whole lines that no other wavefront reads in this sweep (every slot has
// exactly one puller), so it streams past the caches; with c_ix != 0 the
// run straddles a line that the neighbouring wavefront reads too.
template <int I, typename S, bool STREAM = true>
__device__ __forceinline__ Pair<Cmp<S>> load_pull(const S *__restrict__ at) {
    if constexpr (STREAM && cx(I) == 0)
        return Storage<S>::load_stream(at, 0);
    else
        return Storage<S>::load(at, 0);
}

// f_i(x) = slot (i, x - c_i), row-aligned addressing; STREAM: the pulls
// that no other wavefront reads carry the streaming hint
template <typename S, bool STREAM = true, typename T = Cmp<S>>
__device__ __forceinline__ void pull_load_rows(const S *__restrict__ fin, const RowView<S> &rv, T (&f)[2][Q]) {
    const char *base = reinterpret_cast<const char *>(fin);
    Unroll<Q>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const char *row = base + rv.row(-cy(i), -cz(i)) * rv.prow + (size_t)i * RowView<S>::DB;
        const Pair<T> v = load_pull<i, S, STREAM>(reinterpret_cast<const S *>(row + rv.po[1 - cx(i)]));
        f[0][i] = v.x;
        f[1][i] = v.y;
    });
}

// sum_i f_i(x) of both components, row-aligned addressing
template <typename S, bool STREAM = true, typename T = Cmp<S>>
__device__ __forceinline__ void pull_sum_rows(const S *__restrict__ fin, const RowView<S> &rv, T &s0, T &s1) {
    const char *base = reinterpret_cast<const char *>(fin);
    s0 = 0;
    s1 = 0;
    Unroll<Q>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const char *row = base + rv.row(-cy(i), -cz(i)) * rv.prow + (size_t)i * RowView<S>::DB;
        const Pair<T> v = load_pull<i, S, STREAM>(reinterpret_cast<const S *>(row + rv.po[1 - cx(i)]));
        s0 += v.x;
        s1 += v.y;
    });
}

// Tuning macro of the collide sweep (compile-time): LBM_COLLIDE_WAVES is the
// minimum number of wavefronts per SIMD its registers are limited to (0: the
// compiler's choice)
#ifndef LBM_COLLIDE_WAVES
#define LBM_COLLIDE_WAVES 0
#endif
#if LBM_COLLIDE_WAVES > 0
#define LBM_COLLIDE_ATTR __attribute__((amdgpu_waves_per_eu(LBM_COLLIDE_WAVES)))
#else
#define LBM_COLLIDE_ATTR
#endif

// An empty asm statement that takes the values as inputs: loads issued
// before it complete before it, and the compiler cannot sink them into the
// branches that follow, so all of a wavefront's loads are in flight together.
template <typename T, int K>
__device__ __forceinline__ void hold_loads(const T (&v)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) asm volatile("" ::"v"(v[k]));
}

// sum_i f_i(x) of both components (pull form)
template <typename S, typename T = Cmp<S>>
__device__ __forceinline__ void pull_sum(const S *__restrict__ fin, unsigned n, const NbrOffsets &o, T &s0, T &s1) {
    s0 = 0;
    s1 = 0;
    Unroll<Q>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const unsigned src = i == 0 ? n : (unsigned)((int)n + o.template off<opp(i)>());
        const Pair<T> v = load_pop(fin, pidx(0, i, src));
        s0 += v.x;
        s1 += v.y;
    });
}

// ---------------------------------------------------------------------------
// The site update shared by both fluid kernels: BGK collision with the
// velocity shift, Eqs. (2), (3), (6), of a fluid site x (linear index n) whose
// populations are in f and whose neighbour sum of Eq. (4) is acc; f is
// replaced by f*.  Streaming, Eqs. (11), (12), is the caller's store of f*_i
// into slot (i, x); bounce-back at solid neighbours, Eq. (16), is done by the
// link kernels (spheres: the link force sum; walls: the wall-plane kernel),
// which need the density of x and find it in rho_out at boundary sites.
// ---------------------------------------------------------------------------
template <typename M, typename T>
__device__ __forceinline__ void collide_site(const DevParams &P, T (&f)[2][Q], const T (&acc)[2][3], uint32_t inf,
                                             unsigned n, T *__restrict__ rho_out, double &mass0, double &mass1) {
    const T rho0 = (T)P.rho0, irho0 = (T)P.inv_rho0, g = (T)P.g;
    T dr[2], r[2], j[2][3], F[2][3];
    moments(f[0], (T)P.rho_ref[0], dr[0], r[0], j[0][0], j[0][1], j[0][2]);
    moments(f[1], (T)P.rho_ref[1], dr[1], r[1], j[1][0], j[1][1], j[1][2]);
    mass0 += (double)dr[0] + P.rho_ref[0];
    mass1 += (double)dr[1] + P.rho_ref[1];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const T ps = psi_of(r[c], rho0, irho0);
#pragma unroll
        for (int a = 0; a < 3; ++a) F[c][a] = -ps * g * acc[1 - c][a] + r[c] * (T)P.body[a];
    }
    T ueq[2][3];
    eq_velocity<T, M::velocity_mode>(P, r, j, F, ueq);
    if (rho_out && (inf & 0x7fffeu))  // density of a boundary site, read back by the link kernels
        store_pair(rho_out, sidx(0, n), dr[0], dr[1]);
    relax<T, M::eq_order>(f[0], dr[0], r[0], ueq[0][0], ueq[0][1], ueq[0][2], (T)P.inv_tau[0]);
    relax<T, M::eq_order>(f[1], dr[1], r[1], ueq[1][0], ueq[1][1], ueq[1][2], (T)P.inv_tau[1]);
}

// The Shan-Chen force F of a virtual-fluid site is kept for the link
// kernel's sums in the site's own population slots, which carry nothing else
// between the sweep and the link kernel: (Fx, Fy) in slot 0 and (Fz, 0) in
// slot j0, the first direction whose neighbour is not fluid (no bounce-back
// writes it).  This replaces three scattered partial-line stores into a force
// array by values of the sweep's full-lane stores.  It needs the stored type
// to be the arithmetic type (FP32, FP64) and such a direction to exist;
// otherwise the force array is used.  Writer and reader decide alike.
__device__ __forceinline__ int shell_force_slot(uint32_t inf) { return __ffs(inf & 0x7fffeu) - 1; }
template <typename S>
__device__ __forceinline__ bool shell_force_in_slots(uint32_t inf) {
    return std::is_same<S, Cmp<S>>::value && shell_force_slot(inf) > 0;
}
template <typename T>
__device__ __forceinline__ void put_shell_force(T (&f)[2][Q], const T (&F)[3], uint32_t inf) {
    const int j0 = shell_force_slot(inf);
    f[0][0] = F[0];
    f[1][0] = F[1];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        f[0][i] = i == j0 ? F[2] : f[0][i];
        f[1][i] = i == j0 ? (T)0 : f[1][i];
    }
}

// Shan-Chen force of Eq. (4) on a virtual-fluid site, kept for the particle
// sums: Psi of the site is its stored deviation plus Psi(rho_ref) = rho0 - psi_e
template <typename T>
__device__ __forceinline__ void shell_force(const DevParams &P, const T (&own)[2], const T (&acc)[2][3], T (&F)[3]) {
    const T g = (T)P.g;
    const T ps0 = own[0] + (T)(P.rho0 - P.psi_e[0]);
    const T ps1 = own[1] + (T)(P.rho0 - P.psi_e[1]);
#pragma unroll
    for (int a = 0; a < 3; ++a) F[a] = -ps0 * g * acc[1][a] - ps1 * g * acc[0][a];
}

// ---------------------------------------------------------------------------
// deterministic block reductions (blockDim.x == BLOCK)
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double *lds /* >= K * BLOCK / 64 */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NW = BLOCK / 64;
#pragma unroll
    for (int k = 0; k < K; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) lds[k * NW + wave] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += lds[k * NW + w];
        v[k] = t;
    }
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
