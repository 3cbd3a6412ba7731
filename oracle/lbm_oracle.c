/*
 * Plain FP64 CPU oracle: one time step of the two-component Shan-Chen D3Q19
 * lattice Boltzmann fluid with suspended, moving, wettable spheres, as stated in
 * Jansen & Harting, "From Bijels to Pickering emulsions: a lattice Boltzmann
 * study" (arXiv:1004.4414), Secs. II-IV.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this library. The GPU library never links, includes
 * or calls it, and it shares no code, header, table or helper with it.
 *
 * Written to be read against the paper, not to be fast: every step of the
 * method is one plain loop over the lattice, in the order listed in step_once().
 * All floating point is double; build with -ffp-contract=off so that no fused
 * multiply-add changes the rounding of the written expressions.
 *
 * Where the paper is silent or garbled the reading taken is stated at the spot
 * (marked "Reading:").
 *
 * Parity unpinned: the particle colour to contact-angle relation (Sec. V) is an
 * input conversion fitted by the paper; nothing here reproduces that fit.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19
#define NCOMP 2
#define FLUID (-1)
#define WALL_LO (-2)
#define WALL_HI (-3)
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------- */
/* D3Q19 velocity set (Sec. II: "D3Q19 implementation", N = 19 velocities).   */
/* Index 0 is the rest velocity, 1-6 the faces, 7-18 the edges.  The weights  */
/* zeta_i are not printed in the paper; these are the standard D3Q19 weights */
/* 1/3, 1/18, 1/36, pinned by the lattice moment identities in the tests.   */
/* ------------------------------------------------------------------------- */
static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double zeta_of(int i) {
    int n2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
    if (n2 == 0) return 1.0 / 3.0;
    if (n2 == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* index of the opposite velocity, c_opp = -c_i, found by search (once) */
static int opposite(int i) {
    static int table[Q];
    static int ready = 0;
    if (!ready) {
        for (int m = 0; m < Q; ++m) {
            table[m] = -1;
            for (int k = 0; k < Q; ++k)
                if (CV[k][0] == -CV[m][0] && CV[k][1] == -CV[m][1] && CV[k][2] == -CV[m][2]) table[m] = k;
        }
        ready = 1;
    }
    return table[i];
}

static const double CS2 = 1.0 / 3.0; /* c_s = 1/sqrt(3), Sec. II */

typedef struct {
    int32_t nx, ny, nz;
    double tau[2];        /* relaxation time per component, Eq. (2) */
    double g_br;          /* coupling g_rb = g_br, Eq. (4) */
    double rho0;          /* reference density inside Psi, Eq. (5) */
    double w_face, w_edge; /* weights of the neighbour sum in Eq. (4) */
    int32_t velocity_mode; /* 0: common velocity (Shan-Chen), 1: per-component */
    int32_t eq_order;      /* 3 (Eq. (3) as printed) or 2 */
    double rho_init[2];
    double noise_amp;
    uint64_t seed;
    double body_accel[3];  /* test device: uniform acceleration on the fluid */
    int32_t wall_axis;     /* test device: -1 none, else two wall planes */
    double wall_vel[2][3];
    double c0_mass_corr;   /* C_0 of Eq. (31) */
    double k_hertz, lub_hc, lub_hmin;
    int32_t virtual_fluid; /* 1: paper's virtual fluid (Sec. IV); 0: empty particles */
    int32_t lub_mode;      /* 0: Eq. (22) as an explicit force; 1: pair impulses (see move_particles) */
    int32_t force_average; /* 0: this step's fluid force; 1: mean over two steps (see move_particles) */
} orc_params;

typedef struct {
    orc_params p;
    int nx, ny, nz;
    long N;
    double *f[NCOMP];  /* f[c][i*N + n], post-streaming populations at time t */
    double *fs[NCOMP]; /* post-collision populations f* (scratch) */
    double *rho[NCOMP], *j[NCOMP], *F[NCOMP], *psi[NCOMP], *rhov[NCOMP];
    int32_t *owner, *owner_new;
    unsigned char *is_shell;
    /* particles */
    int np, cap;
    double *R, *U, *W;  /* position R(t), velocity U(t-1/2), angular velocity Omega(t-1/2) */
    double *rad, *dens, *color, *mass, *inertia;
    int32_t *prescribed;
    double *Ffl, *Tfl;  /* fluid force / torque of the last step (links + Shan-Chen) */
    double *Fprev, *Tprev; /* fluid force / torque of the step before (force_average) */
    int32_t *have_prev;    /* 1 once a sphere has one */
    double *Ftot, *Ttot; /* total force / torque applied in the last step */
    double *P, *PT;     /* pending impulse / angular impulse from covering / uncovering */
    double wall_force[2][3];
    /* bookkeeping */
    long step;
    int have_M0;
    double M0[NCOMP], Mstep[NCOMP];
    long covered_total, uncovered_total, fallback_total;
    long covered_last, uncovered_last;
    double covered_mass[NCOMP], refill_mass[NCOMP]; /* running totals */
    double wall_mass[NCOMP]; /* running total of the mass the moving-wall term adds */
    int runaway; /* a sphere moved a lattice unit or more in one step (or left the reals) */
} orc_state;

/* ------------------------------------------------------------------------- */
/* lattice geometry                                                           */
/* ------------------------------------------------------------------------- */
static int wrapi(int a, int n) { return ((a % n) + n) % n; }
static long site(const orc_state *s, int x, int y, int z) {
    return ((long)wrapi(z, s->nz) * s->ny + wrapi(y, s->ny)) * s->nx + wrapi(x, s->nx);
}
static void coords(const orc_state *s, long n, int *x, int *y, int *z) {
    *x = (int)(n % s->nx);
    *y = (int)((n / s->nx) % s->ny);
    *z = (int)(n / ((long)s->nx * s->ny));
}
static long neighbour(const orc_state *s, long n, int i, int sign) {
    int x, y, z;
    coords(s, n, &x, &y, &z);
    return site(s, x + sign * CV[i][0], y + sign * CV[i][1], z + sign * CV[i][2]);
}
/* minimum-image displacement along one axis of length L */
static double minimg(double d, double L) {
    while (d > 0.5 * L) d -= L;
    while (d < -0.5 * L) d += L;
    return d;
}
static void cross(const double a[3], const double b[3], double out[3]) {
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

/* ------------------------------------------------------------------------- */
/* SplitMix64 (Steele, Lea, Flood 2014): the k-th output (k = 0, 1, ...) of a */
/* generator seeded with s is mix(s + (k+1)*0x9E3779B97F4A7C15).              */
/* ------------------------------------------------------------------------- */
static uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static double uniform01(uint64_t seed, uint64_t k) {
    return (double)(splitmix64_at(seed, k) >> 11) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------- */
/* Eq. (3): third-order equilibrium (second order when eq_order == 2).       */
/* ------------------------------------------------------------------------- */
static void equilibrium(double rho, const double u[3], int order, double feq[Q]) {
    double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        double bracket = 1.0 + cu / CS2 + (cu * cu) / (2.0 * CS2 * CS2) - u2 / (2.0 * CS2);
        if (order >= 3)
            bracket += (cu * cu * cu) / (6.0 * CS2 * CS2 * CS2) - u2 * cu / (2.0 * CS2 * CS2);
        feq[i] = zeta_of(i) * rho * bracket;
    }
}

/* Eq. (5): effective mass */
static double psi_of(double rho, double rho0) { return rho0 * (1.0 - exp(-rho / rho0)); }

/* neighbour weight W_i of the sum in Eq. (4).  Reading: the paper restricts
 * the sum to the nearest neighbours without naming the set; all 18 non-rest
 * D3Q19 neighbours are used, faces weighted w_face and edges w_edge. */
static double sc_weight(const orc_state *s, int i) {
    int n2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
    if (n2 == 1) return s->p.w_face;
    if (n2 == 2) return s->p.w_edge;
    return 0.0;
}

/* ------------------------------------------------------------------------- */
/* particle discretisation (Sec. III: sites inside the sphere are solid).      */
/* Reading: "inside" is the strict test |x - R| < r, evaluated on positions    */
/* rounded to multiples of 2^-20 so that the classification is exact integer   */
/* arithmetic and independent of the order of floating-point operations.      */
/* ------------------------------------------------------------------------- */
static int64_t fixed20(double v) { return llrint(v * 1048576.0); }

static int inside_sphere(const orc_state *s, int p, int x, int y, int z) {
    const int pos[3] = {x, y, z};
    const int L[3] = {s->nx, s->ny, s->nz};
    int64_t d2 = 0;
    for (int a = 0; a < 3; ++a) {
        int64_t Lq = (int64_t)L[a] << 20;
        int64_t d = ((int64_t)pos[a] << 20) - fixed20(s->R[3 * p + a]);
        while (d > Lq / 2) d -= Lq;
        while (d <= -(Lq / 2)) d += Lq;
        d2 += d * d;
    }
    int64_t rq = fixed20(s->rad[p]);
    return d2 < rq * rq;
}

/* owner map of the current particle positions: walls stay walls, every other
 * site belongs to the lowest-index particle that contains it, else fluid */
static void build_owner_map(const orc_state *s, int32_t *out) {
    for (long n = 0; n < s->N; ++n) out[n] = (s->owner[n] == WALL_LO || s->owner[n] == WALL_HI) ? s->owner[n] : FLUID;
    for (int p = 0; p < s->np; ++p) {
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = (int)floor(s->R[3 * p + a] - s->rad[p]) - 1;
            hi[a] = (int)ceil(s->R[3 * p + a] + s->rad[p]) + 1;
        }
        for (int z = lo[2]; z <= hi[2]; ++z)
            for (int y = lo[1]; y <= hi[1]; ++y)
                for (int x = lo[0]; x <= hi[0]; ++x) {
                    int xw = wrapi(x, s->nx), yw = wrapi(y, s->ny), zw = wrapi(z, s->nz);
                    long n = site(s, xw, yw, zw);
                    if (out[n] == FLUID && inside_sphere(s, p, xw, yw, zw)) out[n] = p;
                }
    }
}

/* ------------------------------------------------------------------------- */
/* creation                                                                   */
/* ------------------------------------------------------------------------- */
orc_state *orc_create(const orc_params *prm) {
    orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
    if (!s) return NULL;
    s->p = *prm;
    s->nx = prm->nx; s->ny = prm->ny; s->nz = prm->nz;
    s->N = (long)s->nx * s->ny * s->nz;
    long N = s->N;
    for (int c = 0; c < NCOMP; ++c) {
        s->f[c] = (double *)calloc((size_t)Q * N, sizeof(double));
        s->fs[c] = (double *)calloc((size_t)Q * N, sizeof(double));
        s->rho[c] = (double *)calloc(N, sizeof(double));
        s->j[c] = (double *)calloc(3 * N, sizeof(double));
        s->F[c] = (double *)calloc(3 * N, sizeof(double));
        s->psi[c] = (double *)calloc(N, sizeof(double));
        s->rhov[c] = (double *)calloc(N, sizeof(double));
    }
    s->owner = (int32_t *)calloc(N, sizeof(int32_t));
    s->owner_new = (int32_t *)calloc(N, sizeof(int32_t));
    s->is_shell = (unsigned char *)calloc(N, 1);
    for (long n = 0; n < N; ++n) {
        int x, y, z;
        coords(s, n, &x, &y, &z);
        int pos[3] = {x, y, z};
        int L[3] = {s->nx, s->ny, s->nz};
        s->owner[n] = FLUID;
        if (prm->wall_axis >= 0 && prm->wall_axis < 3) {
            int a = prm->wall_axis;
            if (pos[a] == 0) s->owner[n] = WALL_LO;
            else if (pos[a] == L[a] - 1) s->owner[n] = WALL_HI;
        }
    }
    /* Initial fluids at random (Sec. VI): rho^c = rho_init^c + noise*(2U-1),
     * U from SplitMix64 at draw index 2n + c; f = equilibrium at rest. */
    for (long n = 0; n < N; ++n) {
        if (s->owner[n] != FLUID) continue;
        for (int c = 0; c < NCOMP; ++c) {
            double U = uniform01(prm->seed, 2 * (uint64_t)n + (uint64_t)c);
            double r = prm->rho_init[c] + prm->noise_amp * (2.0 * U - 1.0);
            for (int i = 0; i < Q; ++i) s->f[c][(long)i * N + n] = zeta_of(i) * r;
        }
    }
    return s;
}

void orc_destroy(orc_state *s) {
    if (!s) return;
    for (int c = 0; c < NCOMP; ++c) {
        free(s->f[c]); free(s->fs[c]); free(s->rho[c]); free(s->j[c]);
        free(s->F[c]); free(s->psi[c]); free(s->rhov[c]);
    }
    free(s->owner); free(s->owner_new); free(s->is_shell);
    free(s->R); free(s->U); free(s->W); free(s->rad); free(s->dens); free(s->color);
    free(s->mass); free(s->inertia); free(s->prescribed); free(s->Ffl); free(s->Tfl);
    free(s->Fprev); free(s->Tprev); free(s->have_prev);
    free(s->Ftot); free(s->Ttot); free(s->P); free(s->PT);
    free(s);
}

/* Add spheres before the first step.  Returns 0, -1 (invalid), -4 (overlap),
 * -5 (called after stepping). */
int orc_add_particles(orc_state *s, int n, const double *pos, const double *vel, const double *omega,
                      const double *radius, const double *density, const double *color,
                      const int32_t *prescribed) {
    if (s->step > 0) return -5;
    if (n < 0) return -1;
    int minL = s->nx < s->ny ? s->nx : s->ny;
    if (s->nz < minL) minL = s->nz;
    const double L[3] = {s->nx, s->ny, s->nz};
    /* spheres need periodic boxes: walls and spheres are not combined */
    if (n > 0 && s->p.wall_axis >= 0) return -1;
    for (int k = 0; k < n; ++k) {
        if (!(radius[k] > 0.0) || radius[k] > 0.25 * minL || !(density[k] > 0.0)) return -1;
        for (int a = 0; a < 3; ++a) {
            if (!(pos[3 * k + a] >= 0.0 && pos[3 * k + a] < L[a])) return -1;
            /* the sphere's bounding box with its neighbour ring, 2 ceil(r) + 7
               sites, must fit in one period of every axis */
            if (2 * (int)ceil(radius[k]) + 7 > (int)L[a]) return -1;
        }
    }
    /* pairwise overlap among new and existing spheres (minimum image) */
    int tot = s->np + n;
    for (int a = 0; a < tot; ++a)
        for (int b = (a + 1 > s->np ? a + 1 : s->np); b < tot; ++b) {
            const double *pa = a < s->np ? &s->R[3 * a] : &pos[3 * (a - s->np)];
            const double *pb = &pos[3 * (b - s->np)];
            double ra = a < s->np ? s->rad[a] : radius[a - s->np];
            double rb = radius[b - s->np];
            double d2 = 0.0;
            for (int ax = 0; ax < 3; ++ax) {
                double d = minimg(pb[ax] - pa[ax], L[ax]);
                d2 += d * d;
            }
            if (d2 <= (ra + rb) * (ra + rb)) return -4;
        }
    if (tot > s->cap) {
        int cap = tot;
        s->R = realloc(s->R, 3 * sizeof(double) * cap); s->U = realloc(s->U, 3 * sizeof(double) * cap);
        s->W = realloc(s->W, 3 * sizeof(double) * cap); s->rad = realloc(s->rad, sizeof(double) * cap);
        s->dens = realloc(s->dens, sizeof(double) * cap); s->color = realloc(s->color, sizeof(double) * cap);
        s->mass = realloc(s->mass, sizeof(double) * cap); s->inertia = realloc(s->inertia, sizeof(double) * cap);
        s->prescribed = realloc(s->prescribed, sizeof(int32_t) * cap);
        s->Ffl = realloc(s->Ffl, 3 * sizeof(double) * cap); s->Tfl = realloc(s->Tfl, 3 * sizeof(double) * cap);
        s->Fprev = realloc(s->Fprev, 3 * sizeof(double) * cap);
        s->Tprev = realloc(s->Tprev, 3 * sizeof(double) * cap);
        s->have_prev = realloc(s->have_prev, sizeof(int32_t) * cap);
        s->Ftot = realloc(s->Ftot, 3 * sizeof(double) * cap); s->Ttot = realloc(s->Ttot, 3 * sizeof(double) * cap);
        s->P = realloc(s->P, 3 * sizeof(double) * cap); s->PT = realloc(s->PT, 3 * sizeof(double) * cap);
        s->cap = cap;
    }
    for (int k = 0; k < n; ++k) {
        int p = s->np + k;
        for (int a = 0; a < 3; ++a) {
            s->R[3 * p + a] = pos[3 * k + a];
            s->U[3 * p + a] = vel[3 * k + a];
            s->W[3 * p + a] = omega[3 * k + a];
            s->Ffl[3 * p + a] = s->Tfl[3 * p + a] = s->Ftot[3 * p + a] = s->Ttot[3 * p + a] = 0.0;
            s->P[3 * p + a] = s->PT[3 * p + a] = 0.0;
        }
        s->rad[p] = radius[k];
        s->dens[p] = density[k];
        s->color[p] = color[k];
        s->prescribed[p] = prescribed[k];
        /* Reading: homogeneous continuum sphere, m = rho_p (4/3) pi r^3, J = (2/5) m r^2 */
        s->mass[p] = density[k] * (4.0 / 3.0) * M_PI * radius[k] * radius[k] * radius[k];
        s->inertia[p] = 0.4 * s->mass[p] * radius[k] * radius[k];
    }
    s->np = tot;
    for (int p = 0; p < tot; ++p) s->have_prev[p] = 0;
    /* the fluid on sites that became solid is removed */
    build_owner_map(s, s->owner_new);
    for (long m = 0; m < s->N; ++m) {
        if (s->owner_new[m] >= 0)
            for (int c = 0; c < NCOMP; ++c)
                for (int i = 0; i < Q; ++i) s->f[c][(long)i * s->N + m] = 0.0;
        s->owner[m] = s->owner_new[m];
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Steps (1)-(4): moments, virtual fluid, effective mass, Shan-Chen force.    */
/* ------------------------------------------------------------------------- */
static void moments_and_forces(orc_state *s) {
    const long N = s->N;
    /* (1) moments on fluid sites, Sec. II: rho^c = rho_0 sum_i f_i with the
     * reading rho_0 = 1 in this definition (rho_0 enters only Eq. (5)), and
     * rho^c u^c = sum_i f_i c_i.  The momentum is summed over opposite pairs
     * (f_i - f_opp) c_i so that a symmetric state gives exactly zero. */
    for (long n = 0; n < N; ++n)
        for (int c = 0; c < NCOMP; ++c) {
            double r = 0.0, jj[3] = {0.0, 0.0, 0.0};
            if (s->owner[n] == FLUID) {
                for (int i = 0; i < Q; ++i) r += s->f[c][(long)i * N + n];
                for (int i = 1; i < Q; ++i) {
                    int o = opposite(i);
                    if (o < i) continue;
                    double d = s->f[c][(long)i * N + n] - s->f[c][(long)o * N + n];
                    for (int a = 0; a < 3; ++a) jj[a] += d * CV[i][a];
                }
            }
            s->rho[c][n] = r;
            for (int a = 0; a < 3; ++a) s->j[c][3 * n + a] = jj[a];
        }
    /* (2) Sec. IV, Eqs. (27), (29), (30): the outermost layer of solid sites
     * inside a particle (reading: particle sites with at least one fluid site
     * among their 18 neighbours) holds a virtual fluid whose density is the
     * mean over its fluid neighbours; the particle colour adds |colour| to the
     * red (colour > 0, component 0) or blue (colour < 0, component 1) density. */
    for (long n = 0; n < N; ++n) {
        s->is_shell[n] = 0;
        s->rhov[0][n] = s->rhov[1][n] = 0.0;
        if (s->owner[n] < 0) continue;
        int cnt = 0;
        double sum[NCOMP] = {0.0, 0.0};
        for (int i = 1; i < Q; ++i) {
            long m = neighbour(s, n, i, +1);
            if (s->owner[m] == FLUID) {
                ++cnt;
                for (int c = 0; c < NCOMP; ++c) sum[c] += s->rho[c][m];
            }
        }
        if (cnt == 0) continue;
        s->is_shell[n] = 1;
        if (!s->p.virtual_fluid) continue;
        for (int c = 0; c < NCOMP; ++c) s->rhov[c][n] = sum[c] / cnt;
        double col = s->color[s->owner[n]];
        if (col > 0.0) s->rhov[0][n] += fabs(col);
        if (col < 0.0) s->rhov[1][n] += fabs(col);
    }
    /* (3) Eq. (5) on fluid and virtual-fluid sites; zero on other solid sites */
    for (long n = 0; n < N; ++n)
        for (int c = 0; c < NCOMP; ++c) {
            if (s->owner[n] == FLUID) s->psi[c][n] = psi_of(s->rho[c][n], s->p.rho0);
            else if (s->is_shell[n]) s->psi[c][n] = psi_of(s->rhov[c][n], s->p.rho0);
            else s->psi[c][n] = 0.0;
        }
    /* (4) Eq. (4) with g_rr = g_bb = 0 and g_rb = g_br:
     *     F^c(x) = -Psi^c(x) g_br sum_i W_i Psi^cbar(x + c_i) c_i,
     * on fluid and virtual-fluid sites; the test-only body acceleration adds
     * rho^c a on fluid sites. */
    for (long n = 0; n < N; ++n)
        for (int c = 0; c < NCOMP; ++c) {
            double Fc[3] = {0.0, 0.0, 0.0};
            if (s->owner[n] == FLUID || s->is_shell[n]) {
                int cb = 1 - c;
                double acc[3] = {0.0, 0.0, 0.0};
                for (int i = 1; i < Q; ++i) {
                    long m = neighbour(s, n, i, +1);
                    double w = sc_weight(s, i) * s->psi[cb][m];
                    for (int a = 0; a < 3; ++a) acc[a] += w * CV[i][a];
                }
                for (int a = 0; a < 3; ++a) Fc[a] = -s->psi[c][n] * s->p.g_br * acc[a];
                if (s->owner[n] == FLUID)
                    for (int a = 0; a < 3; ++a) Fc[a] += s->rho[c][n] * s->p.body_accel[a];
            }
            for (int a = 0; a < 3; ++a) s->F[c][3 * n + a] = Fc[a];
        }
}

/* ------------------------------------------------------------------------- */
/* Step (5): BGK collision with the velocity-shift force, Eqs. (2), (3), (6). */
/* ------------------------------------------------------------------------- */
static void collide(orc_state *s) {
    const long N = s->N;
    for (long n = 0; n < N; ++n) {
        if (s->owner[n] != FLUID) continue;
        double ubar[3] = {0.0, 0.0, 0.0};
        if (s->p.velocity_mode == 0) {
            /* Reading: the bulk fluid velocity in the equilibrium is taken as the
             * Shan-Chen common velocity u' = sum_c (j^c/tau^c) / sum_c (rho^c/tau^c) */
            double den = 0.0, num[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < NCOMP; ++c) {
                den += s->rho[c][n] / s->p.tau[c];
                for (int a = 0; a < 3; ++a) num[a] += s->j[c][3 * n + a] / s->p.tau[c];
            }
            if (den != 0.0)
                for (int a = 0; a < 3; ++a) ubar[a] = num[a] / den;
        }
        for (int c = 0; c < NCOMP; ++c) {
            double r = s->rho[c][n];
            double ueq[3];
            for (int a = 0; a < 3; ++a) {
                double base = ubar[a];
                double shift = 0.0;
                /* Reading: a component of exactly zero density is inert (no
                 * velocity, no shift); any other density, including a
                 * negative one in a violently demixing region, takes Eq. (6)
                 * as written, which keeps the total momentum exact. */
                if (r != 0.0) {
                    if (s->p.velocity_mode == 1) base = s->j[c][3 * n + a] / r;
                    shift = s->p.tau[c] * s->F[c][3 * n + a] / r; /* Eq. (6) */
                } else if (s->p.velocity_mode == 1) {
                    base = 0.0;
                }
                ueq[a] = base + shift;
            }
            double feq[Q];
            equilibrium(r, ueq, s->p.eq_order, feq);
            for (int i = 0; i < Q; ++i) {
                double fi = s->f[c][(long)i * N + n];
                s->fs[c][(long)i * N + n] = fi - (fi - feq[i]) / s->p.tau[c];
            }
        }
    }
}

/* surface velocity of particle p at the point rel (relative to its centre) */
static void particle_surface_velocity(const orc_state *s, int p, const double rel[3], double out[3]) {
    double wxr[3];
    cross(&s->W[3 * p], rel, wxr);
    for (int a = 0; a < 3; ++a) out[a] = s->U[3 * p + a] + wxr[a];
}

/* ------------------------------------------------------------------------- */
/* Step (6): streaming, Eq. (11), with bounce-back on links into solid sites, */
/* Eq. (12), corrected for a moving surface, Eq. (16), and the momentum        */
/* given to the particle, Eqs. (13)-(17).                                      */
/* Readings: the wall term is 2 zeta_i rho (c_i . u_b)/c_s^2 (the paper's     */
/* single 1/6 is the edge-link value; the face links get 1/3); rho is the      */
/* fluid-site density at time t; the transferred momentum uses the reflected   */
/* post-collision population; the lever arm is taken at the link midpoint,     */
/* and the torque is r x F.                                                    */
/* ------------------------------------------------------------------------- */
static void stream_and_bounce(orc_state *s) {
    const long N = s->N;
    const double L[3] = {s->nx, s->ny, s->nz};
    for (int p = 0; p < s->np; ++p)
        for (int a = 0; a < 3; ++a) s->Ffl[3 * p + a] = s->Tfl[3 * p + a] = 0.0;
    for (int w = 0; w < 2; ++w)
        for (int a = 0; a < 3; ++a) s->wall_force[w][a] = 0.0;
    for (long n = 0; n < N; ++n) {
        if (s->owner[n] != FLUID) {
            for (int c = 0; c < NCOMP; ++c)
                for (int i = 0; i < Q; ++i) s->f[c][(long)i * N + n] = 0.0;
            continue;
        }
        int x, y, z;
        coords(s, n, &x, &y, &z);
        for (int c = 0; c < NCOMP; ++c) s->f[c][n] = s->fs[c][n]; /* rest population */
        for (int i = 1; i < Q; ++i) {
            long src = neighbour(s, n, i, -1);
            int own = s->owner[src];
            if (own == FLUID) {
                for (int c = 0; c < NCOMP; ++c) s->f[c][(long)i * N + n] = s->fs[c][(long)i * N + src];
                continue;
            }
            int o = opposite(i);
            double ub[3] = {0.0, 0.0, 0.0};
            double rb[3] = {0.0, 0.0, 0.0};
            if (own >= 0) {
                const double mid[3] = {x - 0.5 * CV[i][0], y - 0.5 * CV[i][1], z - 0.5 * CV[i][2]};
                for (int a = 0; a < 3; ++a) rb[a] = minimg(mid[a] - s->R[3 * own + a], L[a]);
                particle_surface_velocity(s, own, rb, ub);
            } else {
                int wi = own == WALL_LO ? 0 : 1;
                for (int a = 0; a < 3; ++a) ub[a] = s->p.wall_vel[wi][a];
            }
            double cub = CV[i][0] * ub[0] + CV[i][1] * ub[1] + CV[i][2] * ub[2];
            double sum_dp = 0.0; /* momentum given to the solid, along -c_i */
            for (int c = 0; c < NCOMP; ++c) {
                double fo = s->fs[c][(long)o * N + n];
                double wall = 2.0 * zeta_of(i) * s->rho[c][n] * cub / CS2;
                s->f[c][(long)i * N + n] = fo + wall;
                s->wall_mass[c] += wall;
                sum_dp += 2.0 * fo + wall;
            }
            double dp[3] = {-CV[i][0] * sum_dp, -CV[i][1] * sum_dp, -CV[i][2] * sum_dp};
            if (own >= 0) {
                double tq[3];
                cross(rb, dp, tq);
                for (int a = 0; a < 3; ++a) {
                    s->Ffl[3 * own + a] += dp[a];
                    s->Tfl[3 * own + a] += tq[a];
                }
            } else {
                int wi = own == WALL_LO ? 0 : 1;
                for (int a = 0; a < 3; ++a) s->wall_force[wi][a] += dp[a];
            }
        }
    }
}

/* Step (7), Eq. (28): the Shan-Chen force on the virtual fluid of a particle
 * acts on the particle, with the matching torque about its centre. */
static void shan_chen_on_particles(orc_state *s) {
    const long N = s->N;
    const double L[3] = {s->nx, s->ny, s->nz};
    for (long n = 0; n < N; ++n) {
        if (!s->is_shell[n]) continue;
        int p = s->owner[n];
        int x, y, z;
        coords(s, n, &x, &y, &z);
        const double pos[3] = {x, y, z};
        double Fs[3], r[3], tq[3];
        for (int a = 0; a < 3; ++a) {
            Fs[a] = s->F[0][3 * n + a] + s->F[1][3 * n + a];
            r[a] = minimg(pos[a] - s->R[3 * p + a], L[a]);
        }
        cross(r, Fs, tq);
        for (int a = 0; a < 3; ++a) {
            s->Ffl[3 * p + a] += Fs[a];
            s->Tfl[3 * p + a] += tq[a];
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Steps (8)-(9): particle-particle forces, Eqs. (21), (22), and the leap-frog */
/* integration of Eqs. (9), (10).                                              */
/* Readings: K_Hertz is a parameter; the Hertz force is -dV/dr along the      */
/* centre line with 2 r_par generalised to r_a + r_b.  The lubrication force  */
/* is -c rhat [rhat.(u_1-u_2)] with c = 6 pi nu rho_0 (r_a r_b/(r_a+r_b))^2    */
/* (1/h - 1/h_c) for gaps h = |r| - r_a - r_b below h_c, with h clamped at     */
/* h_min; nu is the mean of c_s^2 (tau^c - 1/2).                               */
/* Reading (integration; the paper names a leap-frog and no scheme for this   */
/* velocity-dependent force), two modes:                                     */
/*  lub_mode 0: Eq. (22) as printed, an explicit force: u_1 - u_2 are the     */
/*    latest velocities U(t-1/2), and the force joins every other force in    */
/*    U(t+1/2) = U(t-1/2) + F/m.  For an isolated pair the approach speed     */
/*    becomes w (1 - c (1/m_1 + 1/m_2)): with c (1/m_1 + 1/m_2) > 2, which    */
/*    happens at the h_min clamp for particle densities near the fluid's,     */
/*    it reverses and grows every step.                                      */
/*  lub_mode 1 (default): pair impulses.  With v* the velocities after every  */
/*    other force, w = n.(v*_p - v*_q) the approach speed and k_p the number  */
/*    of lubrication contacts of sphere p, the pair exchanges                */
/*    J = c w / (1 + c (k_p/m_p + k_q/m_q)) along n, equal and opposite.  For */
/*    an isolated pair (k = 1) this is the backward-Euler solution of the     */
/*    pair's lubrication; sharing each sphere's mass among its contacts keeps */
/*    the simultaneous impulses from overshooting.                           */
/* A sphere with prescribed motion counts as infinitely heavy.                */
/* Reading (force_average 1; the paper takes the link coupling from Ladd's    */
/* method and states no such step): the fluid force and torque that enter     */
/* the leap-frog are the mean of this step's and the previous step's, or this */
/* step's alone in a sphere's first step.  The momentum the spheres take from */
/* the fluid over steps 1..T is then the sum of the fluid forces plus half    */
/* the first step's minus half the last step's.                               */
/* ------------------------------------------------------------------------- */
static void move_particles(orc_state *s) {
    const double L[3] = {s->nx, s->ny, s->nz};
    const int np = s->np;
    double nu = 0.0;
    for (int c = 0; c < NCOMP; ++c) nu += CS2 * (s->p.tau[c] - 0.5);
    nu /= NCOMP;
    for (int p = 0; p < np; ++p) {
        const int avg = s->p.force_average && s->have_prev[p];
        for (int a = 0; a < 3; ++a) {
            double ff = s->Ffl[3 * p + a], tf = s->Tfl[3 * p + a];
            if (avg) {
                ff = 0.5 * (ff + s->Fprev[3 * p + a]);
                tf = 0.5 * (tf + s->Tprev[3 * p + a]);
            }
            s->Fprev[3 * p + a] = s->Ffl[3 * p + a];
            s->Tprev[3 * p + a] = s->Tfl[3 * p + a];
            s->Ftot[3 * p + a] = ff + s->P[3 * p + a];
            s->Ttot[3 * p + a] = tf + s->PT[3 * p + a];
        }
        s->have_prev[p] = 1;
    }
    /* Hertz repulsion; lubrication contacts (p < q, unit vector n from p to q) */
    int ncon = 0, capcon = 16;
    int *cp = malloc(sizeof(int) * capcon), *cq = malloc(sizeof(int) * capcon);
    double *cc = malloc(sizeof(double) * capcon), *cn = malloc(sizeof(double) * 3 * capcon);
    for (int p = 0; p < np; ++p)
        for (int q = p + 1; q < np; ++q) {
            double d[3], dist2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                d[a] = minimg(s->R[3 * q + a] - s->R[3 * p + a], L[a]);
                dist2 += d[a] * d[a];
            }
            double dist = sqrt(dist2);
            double rsum = s->rad[p] + s->rad[q];
            if (dist <= 0.0) continue;
            double nh[3] = {d[0] / dist, d[1] / dist, d[2] / dist};
            if (dist < rsum) {
                double fh = 2.5 * s->p.k_hertz * pow(rsum - dist, 1.5);
                for (int a = 0; a < 3; ++a) {
                    s->Ftot[3 * p + a] -= fh * nh[a];
                    s->Ftot[3 * q + a] += fh * nh[a];
                }
            }
            double h = dist - rsum;
            if (s->p.lub_hc > 0.0 && h < s->p.lub_hc) { /* h_c <= 0 switches it off */
                double hh = h < s->p.lub_hmin ? s->p.lub_hmin : h;
                double ared = s->rad[p] * s->rad[q] / rsum;
                if (ncon == capcon) {
                    capcon *= 2;
                    cp = realloc(cp, sizeof(int) * capcon);
                    cq = realloc(cq, sizeof(int) * capcon);
                    cc = realloc(cc, sizeof(double) * capcon);
                    cn = realloc(cn, sizeof(double) * 3 * capcon);
                }
                cp[ncon] = p;
                cq[ncon] = q;
                cc[ncon] = 6.0 * M_PI * nu * s->p.rho0 * ared * ared * (1.0 / hh - 1.0 / s->p.lub_hc);
                for (int a = 0; a < 3; ++a) cn[3 * ncon + a] = nh[a];
                ++ncon;
            }
        }
    if (s->p.lub_mode == 0)
        for (int k = 0; k < ncon; ++k) {
            const int p = cp[k], q = cq[k];
            const double *n = cn + 3 * k;
            double w = 0.0;
            for (int a = 0; a < 3; ++a) w += n[a] * (s->U[3 * p + a] - s->U[3 * q + a]);
            for (int a = 0; a < 3; ++a) {
                s->Ftot[3 * p + a] -= cc[k] * w * n[a];
                s->Ftot[3 * q + a] += cc[k] * w * n[a];
            }
        }
    /* velocities after every other force */
    double *vs = malloc(sizeof(double) * 3 * (size_t)(np > 0 ? np : 1));
    for (int p = 0; p < np; ++p)
        for (int a = 0; a < 3; ++a)
            vs[3 * p + a] = s->U[3 * p + a] + (s->prescribed[p] ? 0.0 : s->Ftot[3 * p + a] / s->mass[p]);
    if (ncon > 0 && s->p.lub_mode != 0) {
        int *kc = calloc((size_t)np, sizeof(int));
        for (int k = 0; k < ncon; ++k) {
            ++kc[cp[k]];
            ++kc[cq[k]];
        }
        double *imp = calloc((size_t)3 * np, sizeof(double));
        for (int k = 0; k < ncon; ++k) {
            const int p = cp[k], q = cq[k];
            const double *n = cn + 3 * k;
            double w = 0.0;
            for (int a = 0; a < 3; ++a) w += n[a] * (vs[3 * p + a] - vs[3 * q + a]);
            const double inv = (s->prescribed[p] ? 0.0 : kc[p] / s->mass[p]) +
                               (s->prescribed[q] ? 0.0 : kc[q] / s->mass[q]);
            const double J = cc[k] * w / (1.0 + cc[k] * inv);
            for (int a = 0; a < 3; ++a) {
                imp[3 * p + a] -= J * n[a];
                imp[3 * q + a] += J * n[a];
            }
        }
        for (int p = 0; p < np; ++p)
            for (int a = 0; a < 3; ++a) {
                s->Ftot[3 * p + a] += imp[3 * p + a];
                if (!s->prescribed[p]) vs[3 * p + a] += imp[3 * p + a] / s->mass[p];
            }
        free(kc);
        free(imp);
    }
    for (int p = 0; p < np; ++p) {
        for (int a = 0; a < 3; ++a) {
            if (!s->prescribed[p]) {
                s->U[3 * p + a] = vs[3 * p + a];
                s->W[3 * p + a] += s->Ttot[3 * p + a] / s->inertia[p];
            }
            /* the map update takes sub-lattice moves per step: a faster or
               non-finite sphere is outside the scheme and stops the run */
            if (!(fabs(s->U[3 * p + a]) < 1.0)) s->runaway = 1;
            double r = s->R[3 * p + a] + s->U[3 * p + a];
            if (r >= L[a]) r -= L[a];
            if (r < 0.0) r += L[a];
            s->R[3 * p + a] = r;
            s->P[3 * p + a] = 0.0;
            s->PT[3 * p + a] = 0.0;
        }
    }
    free(vs);
    free(cp);
    free(cq);
    free(cc);
    free(cn);
}

/* ------------------------------------------------------------------------- */
/* Step (10): the moved particles cover and uncover sites.                     */
/* Covering, Eq. (18): the fluid is removed and its momentum goes to the       */
/* particle (reading: the particle gains +sum_c sum_i f_i c_i of the removed   */
/* populations, with the matching angular impulse).                           */
/* Uncovering, Eqs. (23)-(26), (31): new fluid of density rho_new^c = mean of  */
/* rho^c over the neighbours that are fluid before and after the move, scaled */
/* by the mass correction of Eq. (31), at the equilibrium of the local surface */
/* velocity; the particle loses the created momentum.  Readings: density      */
/* enters f_i once; the impulses are applied in the next step's integration;  */
/* in Eq. (31) Delta rho^c is the fluid mass at the start of this step minus   */
/* that at the start of the first step and N the number of lattice sites.     */
/* ------------------------------------------------------------------------- */
static void update_map(orc_state *s) {
    const long N = s->N;
    const double L[3] = {s->nx, s->ny, s->nz};
    build_owner_map(s, s->owner_new);
    s->covered_last = s->uncovered_last = 0;
    /* covering */
    for (long n = 0; n < N; ++n) {
        int q = s->owner_new[n];
        if (s->owner[n] != FLUID || q < 0) continue;
        int x, y, z;
        coords(s, n, &x, &y, &z);
        const double pos[3] = {x, y, z};
        double mom[3] = {0.0, 0.0, 0.0}, r[3], tq[3];
        for (int c = 0; c < NCOMP; ++c)
            for (int i = 0; i < Q; ++i) {
                double fi = s->f[c][(long)i * N + n];
                for (int a = 0; a < 3; ++a) mom[a] += fi * CV[i][a];
                s->covered_mass[c] += fi;
                s->f[c][(long)i * N + n] = 0.0;
            }
        for (int a = 0; a < 3; ++a) r[a] = minimg(pos[a] - s->R[3 * q + a], L[a]);
        cross(r, mom, tq);
        for (int a = 0; a < 3; ++a) {
            s->P[3 * q + a] += mom[a];
            s->PT[3 * q + a] += tq[a];
        }
        ++s->covered_last;
    }
    /* uncovering: densities from the neighbours first (Jacobi), then refill */
    double sumrinit = s->p.rho_init[0] + s->p.rho_init[1];
    for (long n = 0; n < N; ++n) {
        int p = s->owner[n];
        if (p < 0 || s->owner_new[n] != FLUID) continue;
        double rbar[NCOMP] = {0.0, 0.0};
        int cnt = 0;
        for (int i = 1; i < Q; ++i) {
            long m = neighbour(s, n, i, +1);
            if (s->owner[m] != FLUID || s->owner_new[m] != FLUID) continue;
            ++cnt;
            for (int c = 0; c < NCOMP; ++c) {
                double r = 0.0;
                for (int k = 0; k < Q; ++k) r += s->f[c][(long)k * N + m];
                rbar[c] += r;
            }
        }
        double rnew[NCOMP];
        for (int c = 0; c < NCOMP; ++c) {
            if (cnt > 0) rnew[c] = rbar[c] / cnt;
            else rnew[c] = s->p.rho_init[c];
            if (s->p.c0_mass_corr != 0.0 && s->p.rho_init[c] > 0.0) {
                double dM = s->Mstep[c] - s->M0[c];
                rnew[c] *= 1.0 - s->p.c0_mass_corr * (sumrinit / s->p.rho_init[c]) * dM / (double)N;
            }
        }
        if (cnt == 0) ++s->fallback_total;
        int x, y, z;
        coords(s, n, &x, &y, &z);
        const double pos[3] = {x, y, z};
        double r[3], us[3], mom[3], tq[3];
        for (int a = 0; a < 3; ++a) r[a] = minimg(pos[a] - s->R[3 * p + a], L[a]);
        particle_surface_velocity(s, p, r, us);
        for (int c = 0; c < NCOMP; ++c) {
            double feq[Q];
            equilibrium(rnew[c], us, s->p.eq_order, feq);
            /* written after all means above are taken: the means read only
             * sites that are fluid before and after, never an uncovered site */
            for (int i = 0; i < Q; ++i) s->fs[c][(long)i * N + n] = feq[i];
            s->refill_mass[c] += rnew[c];
        }
        for (int a = 0; a < 3; ++a) mom[a] = (rnew[0] + rnew[1]) * us[a];
        cross(r, mom, tq);
        for (int a = 0; a < 3; ++a) {
            s->P[3 * p + a] -= mom[a];
            s->PT[3 * p + a] -= tq[a];
        }
        ++s->uncovered_last;
    }
    /* commit the refilled populations (staged in fs, which is free now) */
    for (long n = 0; n < N; ++n) {
        if (s->owner[n] >= 0 && s->owner_new[n] == FLUID)
            for (int c = 0; c < NCOMP; ++c)
                for (int i = 0; i < Q; ++i) s->f[c][(long)i * N + n] = s->fs[c][(long)i * N + n];
    }
    for (long n = 0; n < N; ++n) s->owner[n] = s->owner_new[n];
    s->covered_total += s->covered_last;
    s->uncovered_total += s->uncovered_last;
}

static void step_once(orc_state *s) {
    moments_and_forces(s); /* (1)-(4) */
    for (int c = 0; c < NCOMP; ++c) {
        double M = 0.0;
        for (long n = 0; n < s->N; ++n) M += s->rho[c][n];
        s->Mstep[c] = M;
        if (!s->have_M0) s->M0[c] = M;
    }
    s->have_M0 = 1;
    collide(s);                /* (5) */
    stream_and_bounce(s);      /* (6) */
    shan_chen_on_particles(s); /* (7) */
    move_particles(s);         /* (8)-(9) */
    update_map(s);             /* (10) */
    ++s->step;
}

/* 0, or -1 once a sphere has run away (the state is then left as it is) */
int orc_step(orc_state *s, int nsteps) {
    for (int k = 0; k < nsteps && !s->runaway; ++k) step_once(s);
    return s->runaway ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* accessors                                                                  */
/* ------------------------------------------------------------------------- */
/* populations, layout [c][i][z][y][x] */
void orc_get_populations(const orc_state *s, double *out) {
    for (int c = 0; c < NCOMP; ++c) memcpy(out + (size_t)c * Q * s->N, s->f[c], sizeof(double) * Q * s->N);
}
/* values on non-fluid sites are ignored (kept zero) */
void orc_set_populations(orc_state *s, const double *in) {
    for (int c = 0; c < NCOMP; ++c)
        for (int i = 0; i < Q; ++i)
            for (long n = 0; n < s->N; ++n)
                s->f[c][(long)i * s->N + n] = s->owner[n] == FLUID ? in[((size_t)c * Q + i) * s->N + n] : 0.0;
}

/* Observables of the current state: rho^c [2][N], j^c [2][N][3], F^c [2][N][3]
 * (Shan-Chen plus body force, on fluid and virtual-fluid sites) and the
 * physical mixture velocity of Eq. (7), reading it as
 * u = sum_c (j^c + F^c/2) / sum_c rho^c  [N][3] (zero off fluid sites). */
void orc_get_fields(orc_state *s, double *rho, double *j, double *F, double *u) {
    moments_and_forces(s);
    const long N = s->N;
    for (int c = 0; c < NCOMP; ++c) {
        if (rho) memcpy(rho + (size_t)c * N, s->rho[c], sizeof(double) * N);
        if (j) memcpy(j + (size_t)c * 3 * N, s->j[c], sizeof(double) * 3 * N);
        if (F) memcpy(F + (size_t)c * 3 * N, s->F[c], sizeof(double) * 3 * N);
    }
    if (u)
        for (long n = 0; n < N; ++n) {
            double den = s->rho[0][n] + s->rho[1][n];
            for (int a = 0; a < 3; ++a) {
                double num = 0.0;
                for (int c = 0; c < NCOMP; ++c) num += s->j[c][3 * n + a] + 0.5 * s->F[c][3 * n + a];
                u[3 * n + a] = (s->owner[n] == FLUID && den > 0.0) ? num / den : 0.0;
            }
        }
}

/* virtual-fluid densities [2][N] of the current state (zero off the shell) */
void orc_get_virtual_density(orc_state *s, double *out) {
    moments_and_forces(s);
    for (int c = 0; c < NCOMP; ++c) memcpy(out + (size_t)c * s->N, s->rhov[c], sizeof(double) * s->N);
}

void orc_get_owner(const orc_state *s, int32_t *out) { memcpy(out, s->owner, sizeof(int32_t) * s->N); }

int orc_num_particles(const orc_state *s) { return s->np; }

/* per particle, 27 doubles: R[3] U[3] W[3] Ffluid[3] Tfluid[3] Ftotal[3]
 * Ttotal[3] P[3] PT[3] */
void orc_get_particles(const orc_state *s, double *out) {
    for (int p = 0; p < s->np; ++p) {
        double *o = out + 27 * p;
        for (int a = 0; a < 3; ++a) {
            o[0 + a] = s->R[3 * p + a];
            o[3 + a] = s->U[3 * p + a];
            o[6 + a] = s->W[3 * p + a];
            o[9 + a] = s->Ffl[3 * p + a];
            o[12 + a] = s->Tfl[3 * p + a];
            o[15 + a] = s->Ftot[3 * p + a];
            o[18 + a] = s->Ttot[3 * p + a];
            o[21 + a] = s->P[3 * p + a];
            o[24 + a] = s->PT[3 * p + a];
        }
    }
}

/* overwrite the kinematic state R, U, W and the pending impulses P, PT
 * (per particle 15 doubles) and rebuild the solid map without touching the
 * fluid; for loading a shared state */
/* Test device: give every sphere a previous step's fluid force and torque
 * (6 doubles per sphere: force, torque), as if it had stepped with them, so
 * that a state taken from a run with force_average 1 continues that run. */
void orc_set_previous_fluid_force(orc_state *s, const double *in) {
    for (int p = 0; p < s->np; ++p) {
        for (int a = 0; a < 3; ++a) {
            s->Fprev[3 * p + a] = in[6 * p + a];
            s->Tprev[3 * p + a] = in[6 * p + 3 + a];
        }
        s->have_prev[p] = 1;
    }
}

void orc_set_particle_state(orc_state *s, const double *in) {
    for (int p = 0; p < s->np; ++p)
        for (int a = 0; a < 3; ++a) {
            s->R[3 * p + a] = in[15 * p + 0 + a];
            s->U[3 * p + a] = in[15 * p + 3 + a];
            s->W[3 * p + a] = in[15 * p + 6 + a];
            s->P[3 * p + a] = in[15 * p + 9 + a];
            s->PT[3 * p + a] = in[15 * p + 12 + a];
        }
    for (int p = 0; p < s->np; ++p) s->have_prev[p] = 0;
    build_owner_map(s, s->owner_new);
    for (long n = 0; n < s->N; ++n) s->owner[n] = s->owner_new[n];
}

/* number of bounce-back links (fluid x, direction i with x - c_i solid) and of
 * virtual-fluid sites per particle, on the current map */
void orc_particle_counts(const orc_state *s, int32_t *links, int32_t *shell) {
    for (int p = 0; p < s->np; ++p) links[p] = shell[p] = 0;
    for (long n = 0; n < s->N; ++n) {
        int own = s->owner[n];
        if (own == FLUID) {
            for (int i = 1; i < Q; ++i) {
                int o = s->owner[neighbour(s, n, i, -1)];
                if (o >= 0) ++links[o];
            }
        } else if (own >= 0) {
            for (int i = 1; i < Q; ++i)
                if (s->owner[neighbour(s, n, i, +1)] == FLUID) {
                    ++shell[own];
                    break;
                }
        }
    }
}

/* running totals per component of the mass removed by covering (out[0..1]),
 * created by refilling (out[2..3]) and added by the moving-wall term of the
 * bounce-back (out[4..5]) */
void orc_event_mass(const orc_state *s, double *out) {
    for (int c = 0; c < NCOMP; ++c) {
        out[c] = s->covered_mass[c];
        out[2 + c] = s->refill_mass[c];
        out[4 + c] = s->wall_mass[c];
    }
}

/* [0] step, [1] covered total, [2] uncovered total, [3] refills without
 * fluid neighbours, [4] covered in the last step, [5] uncovered in the last */
void orc_counts(const orc_state *s, int64_t *out) {
    out[0] = s->step;
    out[1] = s->covered_total;
    out[2] = s->uncovered_total;
    out[3] = s->fallback_total;
    out[4] = s->covered_last;
    out[5] = s->uncovered_last;
}

/* [0..1] fluid mass per component, [2..4] fluid momentum, [5..7] particle
 * momentum sum m U, [8..10] pending impulses, [11..13] force on the walls in
 * the last step */
void orc_sums(const orc_state *s, double *out) {
    for (int k = 0; k < 14; ++k) out[k] = 0.0;
    for (long n = 0; n < s->N; ++n) {
        if (s->owner[n] != FLUID) continue;
        for (int c = 0; c < NCOMP; ++c)
            for (int i = 0; i < Q; ++i) {
                double fi = s->f[c][(long)i * s->N + n];
                out[c] += fi;
                for (int a = 0; a < 3; ++a) out[2 + a] += fi * CV[i][a];
            }
    }
    for (int p = 0; p < s->np; ++p)
        for (int a = 0; a < 3; ++a) {
            out[5 + a] += s->mass[p] * s->U[3 * p + a];
            out[8 + a] += s->P[3 * p + a];
        }
    for (int a = 0; a < 3; ++a) out[11 + a] = s->wall_force[0][a] + s->wall_force[1][a];
}

/* lattice tables for the identity checks: c [19][3], zeta [19], opp [19] */
void orc_lattice(int32_t *c, double *zeta, int32_t *opp) {
    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = CV[i][a];
        zeta[i] = zeta_of(i);
        opp[i] = opposite(i);
    }
}

void orc_equilibrium(double rho, double ux, double uy, double uz, int order, double *out) {
    const double u[3] = {ux, uy, uz};
    equilibrium(rho, u, order, out);
}

double orc_psi(double rho, double rho0) { return psi_of(rho, rho0); }

/* kinematic viscosity of Sec. II, nu = c_s^2 (tau - 1/2), and c_s^2 */
double orc_viscosity(double tau) { return CS2 * (tau - 0.5); }
double orc_cs2(void) { return CS2; }

double orc_uniform01(uint64_t seed, uint64_t k) { return uniform01(seed, k); }
