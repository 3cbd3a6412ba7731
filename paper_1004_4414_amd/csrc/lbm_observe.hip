// Analysis observables off the time-step path: the lateral domain size L(t)
// of Sec. VI (Eqs. (33)-(35)) and order-parameter profiles for the contact
// angle of Sec. V (Eq. (32)).
//
// The order parameter phi = rho_r - rho_b (Sec. II) is taken on fluid sites
// and 0 on solid ones.  For L_i only 1-D transforms along axis i are needed:
// with g(k_i; other coordinates) the DFT of phi' = phi - <phi> along i,
//   sum_k k_i^2 |phi'_k|^2 = (N / n_i) sum_lines sum_{k_i} k_i^2 |g|^2   and
//   sum_k |phi'_k|^2       = N sum_x phi'^2                              ,
// (Parseval over the two other axes), so
//   <k_i^2> = sum_lines sum_{k_i} k_i^2 |g|^2 / (n_i sum_x phi'^2),
// with k_i = 2 pi m / n_i, |m| <= n_i / 2.  Each line is transformed directly
// in FP64 from a twiddle table in LDS (one block per line).
#include <algorithm>
#include <cmath>
#include <mutex>

#include "lbm_handle.h"

namespace lbm {

constexpr int MAX_DFT = 2048;  // longest axis the line transform handles

// phi on fluid sites (0 elsewhere) from the post-streaming populations
template <typename S>
__global__ __launch_bounds__(BLOCK) void k_phi(DevParams P, const S *__restrict__ f, const uint32_t *__restrict__ info,
                                               double *__restrict__ phi) {
    using T = Cmp<S>;
    unsigned n;
    int x, y, z;
    if (!dense_site(P, n, x, y, z)) return;
    double v = 0.0;
    if (site_class(info[n]) == CLS_FLUID) {
        T d0, d1;
        pull_sum(f, n, NbrOffsets(P, x, y, z), d0, d1);
        v = ((double)d0 + P.rho_ref[0]) - ((double)d1 + P.rho_ref[1]);
    }
    phi[n] = v;
}

// per-block sums of phi and phi^2 (fixed order)
__global__ __launch_bounds__(BLOCK) void k_phi_sums(const double *__restrict__ phi, long long N, double mean,
                                                    double *__restrict__ partial) {
    __shared__ double lds[2 * (BLOCK / 64)];
    const long long k = (long long)blockIdx.x * BLOCK + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (k < N) {
        const double d = phi[k] - mean;
        v[0] = phi[k];
        v[1] = d * d;
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = v[0];
        partial[2 * blockIdx.x + 1] = v[1];
    }
}

// sum_{k} k^2 |g(k)|^2 of the line transform of phi' along `axis`; one block
// per line, lines numbered by the two other coordinates
__global__ __launch_bounds__(BLOCK) void k_line_moment(DevParams P, const double *__restrict__ phi, double mean,
                                                       int axis, double *__restrict__ partial) {
    __shared__ double line[MAX_DFT], cs[MAX_DFT], sn[MAX_DFT];
    __shared__ double lds[BLOCK / 64];
    const int L[3] = {P.nx, P.ny, P.nz};
    const int n = L[axis];
    const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;  // the two other axes
    const int u = (int)(blockIdx.x % (unsigned)L[a1]), w = (int)(blockIdx.x / (unsigned)L[a1]);
    const long long stride = axis == 0 ? 1 : (axis == 1 ? (long long)P.nx : (long long)P.nx * P.ny);
    int c[3];
    c[axis] = 0;
    c[a1] = u;
    c[a2] = w;
    const long long base = ((long long)c[2] * P.ny + c[1]) * P.nx + c[0];
    for (int x = threadIdx.x; x < n; x += BLOCK) {
        line[x] = phi[base + x * stride] - mean;
        double s, co;
        sincospi(2.0 * x / n, &s, &co);
        cs[x] = co;
        sn[x] = s;
    }
    __syncthreads();
    double acc = 0.0;
    for (int j = threadIdx.x; j < n; j += BLOCK) {
        double re = 0.0, im = 0.0;
        int idx = 0;  // (j x) mod n
        for (int x = 0; x < n; ++x) {
            re += line[x] * cs[idx];
            im -= line[x] * sn[idx];
            idx += j;
            if (idx >= n) idx -= n;
        }
        const int m = j <= n / 2 ? j : n - j;
        const double k = 2.0 * M_PI * m / n;
        acc += k * k * (re * re + im * im);
    }
    double v[1] = {acc};
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

// plane averages of phi along `axis` (one block per plane, fixed order)
__global__ __launch_bounds__(BLOCK) void k_phi_profile(DevParams P, const double *__restrict__ phi, int axis,
                                                       double *__restrict__ out) {
    __shared__ double lds[BLOCK / 64];
    const int L[3] = {P.nx, P.ny, P.nz};
    const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
    const long long plane = (long long)L[a1] * L[a2];
    double acc = 0.0;
    for (long long k = threadIdx.x; k < plane; k += BLOCK) {
        int c[3];
        c[axis] = (int)blockIdx.x;
        c[a1] = (int)(k % L[a1]);
        c[a2] = (int)(k / L[a1]);
        acc += phi[((long long)c[2] * P.ny + c[1]) * P.nx + c[0]];
    }
    double v[1] = {acc};
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = v[0] / (double)plane;
}

// The plane averages of k_phi + k_phi_profile computed straight from the
// populations, without the phi array: each site's value is formed as k_phi
// forms it and the sums run in the same order, so the results are bitwise
// those of lb_order_parameter_profile.
template <typename S>
__global__ __launch_bounds__(BLOCK) void k_phi_profile_direct(DevParams P, const S *__restrict__ f,
                                                              const uint32_t *__restrict__ info, int axis,
                                                              double *__restrict__ out) {
    using T = Cmp<S>;
    __shared__ double lds[BLOCK / 64];
    const int L[3] = {P.nx, P.ny, P.nz};
    const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
    const long long plane = (long long)L[a1] * L[a2];
    double acc = 0.0;
    for (long long k = threadIdx.x; k < plane; k += BLOCK) {
        int c[3];
        c[axis] = (int)blockIdx.x;
        c[a1] = (int)(k % L[a1]);
        c[a2] = (int)(k / L[a1]);
        const unsigned n = (unsigned)(((long long)c[2] * P.ny + c[1]) * P.nx + c[0]);
        double v = 0.0;
        if (site_class(info[n]) == CLS_FLUID) {
            T d0, d1;
            pull_sum(f, n, NbrOffsets(P, c[0], c[1], c[2]), d0, d1);
            v = ((double)d0 + P.rho_ref[0]) - ((double)d1 + P.rho_ref[1]);
        }
        acc += v;
    }
    double v[1] = {acc};
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = v[0] / (double)plane;
}

// Device scratch of lb_order_parameter_profile_noalloc: one plane average per
// plane, MAX_DFT planes (16 KiB), resident on every device the library runs
// on until the process ends.  In host code `scratch` is only a symbol: its
// device address (one per device) comes from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[MAX_DFT];
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[MAX_DEVICES];

// the address of `scratch` on device dev (current), looked up once per device
static double *scratch_address(int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        double *ptr = nullptr;
        LB_HIP_CHECK(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

static double *phi_buffer(lb_handle *h) {
    if (!h->phi) h->phi = (double *)dev_alloc(h, sizeof(double) * (size_t)h->N);
    return h->phi;
}

static void launch_phi(lb_handle *h) {
    const unsigned nb = (unsigned)((h->N + BLOCK - 1) / BLOCK);
    double *phi = phi_buffer(h);
    with_storage(h->prm, [&](auto tag) {
        using S = typename decltype(tag)::type;
        k_phi<S><<<nb, BLOCK, 0, h->stream>>>(h->dp, (const S *)h->f[h->cur], h->info, phi);
    });
    LB_HIP_CHECK(hipGetLastError());
}

}  // namespace lbm

using namespace lbm;

extern "C" {

int lb_domain_size(lb_handle *h, double L_out[3]) {
    if (!h || !L_out) return LB_EINVAL;
    const int L[3] = {h->prm.nx, h->prm.ny, h->prm.nz};
    for (int a = 0; a < 3; ++a)
        if (L[a] > MAX_DFT) {
            h->err = "an axis is longer than the line transform handles (2048)";
            return LB_EINVAL;
        }
    try {
        settle_bounces(h);
        launch_phi(h);
        const unsigned nb = (unsigned)((h->N + BLOCK - 1) / BLOCK);
        std::vector<double> part(2 * (size_t)nb);
        const int Lmin = std::min(L[0], std::min(L[1], L[2]));
        double *dpart = (double *)dev_alloc(h, sizeof(double) * std::max<size_t>(2 * (size_t)nb, (size_t)(h->N / Lmin)));
        // <phi>
        k_phi_sums<<<nb, BLOCK, 0, h->stream>>>(h->phi, h->N, 0.0, dpart);
        LB_HIP_CHECK(hipGetLastError());
        LB_HIP_CHECK(hipMemcpyAsync(part.data(), dpart, part.size() * 8, hipMemcpyDeviceToHost, h->stream));
        LB_HIP_CHECK(hipStreamSynchronize(h->stream));
        double sum = 0.0;
        for (unsigned b = 0; b < nb; ++b) sum += part[2 * b];
        const double mean = sum / (double)h->N;
        // sum phi'^2
        k_phi_sums<<<nb, BLOCK, 0, h->stream>>>(h->phi, h->N, mean, dpart);
        LB_HIP_CHECK(hipGetLastError());
        LB_HIP_CHECK(hipMemcpyAsync(part.data(), dpart, part.size() * 8, hipMemcpyDeviceToHost, h->stream));
        LB_HIP_CHECK(hipStreamSynchronize(h->stream));
        double var = 0.0;
        for (unsigned b = 0; b < nb; ++b) var += part[2 * b + 1];
        for (int a = 0; a < 3; ++a) {
            const long long lines = h->N / L[a];
            k_line_moment<<<(unsigned)lines, BLOCK, 0, h->stream>>>(h->dp, h->phi, mean, a, dpart);
            LB_HIP_CHECK(hipGetLastError());
            std::vector<double> lp((size_t)lines);
            LB_HIP_CHECK(hipMemcpyAsync(lp.data(), dpart, lp.size() * 8, hipMemcpyDeviceToHost, h->stream));
            LB_HIP_CHECK(hipStreamSynchronize(h->stream));
            double num = 0.0;
            for (double v : lp) num += v;
            const double k2 = var > 0.0 ? num / ((double)L[a] * var) : 0.0;
            L_out[a] = k2 > 0.0 ? 2.0 * M_PI / std::sqrt(k2) : INFINITY;
        }
        dev_free(h, dpart);
    } catch (const HipFailure &e) {
        h->err = e.what;
        return LB_EDEVICE;
    } catch (const std::bad_alloc &) {
        h->err = "device allocation failed";
        return LB_ENOMEM;
    }
    return LB_OK;
}

int lb_order_parameter_profile(lb_handle *h, int32_t axis, double *out) {
    if (!h || !out || axis < 0 || axis > 2) return LB_EINVAL;
    const int L[3] = {h->prm.nx, h->prm.ny, h->prm.nz};
    try {
        settle_bounces(h);
        launch_phi(h);
        double *d = (double *)dev_alloc(h, sizeof(double) * (size_t)L[axis]);
        k_phi_profile<<<(unsigned)L[axis], BLOCK, 0, h->stream>>>(h->dp, h->phi, axis, d);
        LB_HIP_CHECK(hipGetLastError());
        LB_HIP_CHECK(hipMemcpyAsync(out, d, sizeof(double) * L[axis], hipMemcpyDeviceToHost, h->stream));
        LB_HIP_CHECK(hipStreamSynchronize(h->stream));
        dev_free(h, d);
    } catch (const HipFailure &e) {
        h->err = e.what;
        return LB_EDEVICE;
    } catch (const std::bad_alloc &) {
        h->err = "device allocation failed";
        return LB_ENOMEM;
    }
    return LB_OK;
}

int lb_order_parameter_profile_noalloc(lb_handle *h, int32_t axis, double *out) {
    if (!h || !out || axis < 0 || axis > 2) return LB_EINVAL;
    const int L[3] = {h->prm.nx, h->prm.ny, h->prm.nz};
    if (L[axis] > MAX_DFT) {
        h->err = "the profile axis is longer than the scratch holds (2048 planes)";
        return LB_EINVAL;
    }
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) {
        (void)hipGetLastError();
        h->err = "hipGetDevice failed";
        return LB_EDEVICE;
    }
    if (h->device < 0 || h->device >= MAX_DEVICES) {
        h->err = "device index beyond the scratch table";
        return LB_EINVAL;
    }
    try {
        if (cur != h->device) LB_HIP_CHECK(hipSetDevice(h->device));
        settle_bounces(h);
        double *d = scratch_address(h->device);
        with_storage(h->prm, [&](auto tag) {
            using S = typename decltype(tag)::type;
            k_phi_profile_direct<S><<<(unsigned)L[axis], BLOCK, 0, h->stream>>>(h->dp, (const S *)h->f[h->cur],
                                                                              h->info, axis, d);
        });
        LB_HIP_CHECK(hipGetLastError());
        LB_HIP_CHECK(hipMemcpyAsync(out, d, sizeof(double) * L[axis], hipMemcpyDeviceToHost, h->stream));
        LB_HIP_CHECK(hipStreamSynchronize(h->stream));
        if (cur != h->device) LB_HIP_CHECK(hipSetDevice(cur));
    } catch (const HipFailure &e) {
        (void)hipSetDevice(cur);
        h->err = e.what;
        return LB_EDEVICE;
    }
    return LB_OK;
}

}  // extern "C"
