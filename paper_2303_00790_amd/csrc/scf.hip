// Self-consistent field pieces on gfx950 (all FP64): density, PZ81 LDA,
// Hartree potential by CG on the FD Laplacian with multipole boundary
// values, the superposition-of-atoms start density, Anderson mixing, the
// self-consistent residual error, the Harris-Foulkes energy, and one SCF step.
//
// Paper (computational details): LDA in the Ceperley-Alder / Perdew-Zunger
// form; four ChFSI iterations in the first SCF step and one per later step;
// convergence when the SRE -- the square root of the density-weighted
// integral of the squared difference of the last two potentials -- is below
// 1e-4 Ry.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>

#include "internal.hpp"
#include "kernels.hpp"

namespace chf {

constexpr double kPi = 3.14159265358979323846;

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// density: rho[row] = (2 / h^3) sum_{i < n_occ} X[row][i]^2, one wave per row
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) density_kernel(int64_t n_rows, const T* __restrict__ X, int64_t ldx, int n_occ,
                                                      double scale, double* __restrict__ rho) {
    const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n_rows) return;
    const T* xr = X + row * ldx;
    double acc = 0.0;
    for (int i = lane; i < n_occ; i += 64) {
        const double v = double(xr[i]);
        acc += v * v;
    }
    acc = wave_sum(acc);
    if (lane == 0) rho[row] = scale * acc;
}

// ---------------------------------------------------------------------------
// LDA (Perdew-Zunger parametrisation of Ceperley-Alder, unpolarised)
//   r_s = (3 / (4 pi rho))^(1/3),  eps_x = -(3/4) (9 / (4 pi^2))^(1/3) / r_s
//   r_s >= 1: eps_c = g / (1 + b1 sqrt(r_s) + b2 r_s)
//   r_s <  1: eps_c = A ln r_s + B + C r_s ln r_s + D r_s
//   v_xc = eps_xc - (r_s / 3) d eps_xc / d r_s ;  0 where rho < 1e-14
// ---------------------------------------------------------------------------
__global__ void lda_kernel(int64_t n, const double* __restrict__ rho, double* __restrict__ exc,
                           double* __restrict__ vxc) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double r = rho[i];
    if (!(r >= 1e-14)) {
        if (exc) exc[i] = 0.0;
        vxc[i] = 0.0;
        return;
    }
    const double cx = 0.75 * cbrt(9.0 / (4.0 * kPi * kPi));
    const double rs = cbrt(3.0 / (4.0 * kPi * r));
    double ec, dec;
    if (rs >= 1.0) {
        const double g = -0.1423, b1 = 1.0529, b2 = 0.3334;
        const double sq = sqrt(rs);
        const double den = 1.0 + b1 * sq + b2 * rs;
        ec = g / den;
        dec = -g * (0.5 * b1 / sq + b2) / (den * den);
    } else {
        const double A = 0.0311, B = -0.048, Cc = 0.0020, D = -0.0116;
        const double lr = log(rs);
        ec = A * lr + B + Cc * rs * lr + D * rs;
        dec = A / rs + Cc * (lr + 1.0) + D;
    }
    const double ex = -cx / rs, dex = cx / (rs * rs);
    if (exc) exc[i] = ex + ec;
    vxc[i] = (ex + ec) - rs / 3.0 * (dex + dec);
}

// ---------------------------------------------------------------------------
// Hartree: exterior values from Cartesian multipole moments up to order 4,
// contracted through the Legendre expansion of 1/|r - r'| (valid for
// |r| > |r'|):  V(r) = sum_l sum_p q_p |r|^-(2l+1) |r|^l |r_p|^l P_l(cos g).
// Moments: M[a][b][c] = h^3 sum_p rho_p x^a y^b z^c, a + b + c <= 4.
// ---------------------------------------------------------------------------
constexpr int kNMom = 35;

// exponents (a, b, c) of the Cartesian moments x^a y^b z^c, a + b + c <= 4,
// by order, built at compile time into constant memory (every device gets
// the table with the code object)
struct MomExp {
    int e[kNMom][3];
};
constexpr MomExp make_mom_exponents() {
    MomExp t{};
    int k = 0;
    for (int n = 0; n <= 4; ++n)
        for (int a = n; a >= 0; --a)
            for (int b = n - a; b >= 0; --b) {
                t.e[k][0] = a;
                t.e[k][1] = b;
                t.e[k][2] = n - a - b;
                ++k;
            }
    return t;
}
__constant__ MomExp c_mom = make_mom_exponents();

__global__ void __launch_bounds__(256) moments_kernel(int64_t n_rows, const int32_t* __restrict__ ijk4, double h,
                                                      const double* __restrict__ rho, double* __restrict__ part) {
    __shared__ double sh[256];
    double acc[kNMom];
    for (int m = 0; m < kNMom; ++m) acc[m] = 0.0;
    for (int64_t row = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; row < n_rows;
         row += int64_t(gridDim.x) * blockDim.x) {
        if (!ijk4[4 * row + 3]) continue;
        const double q = rho[row];
        const double x = ijk4[4 * row] * h, y = ijk4[4 * row + 1] * h, z = ijk4[4 * row + 2] * h;
        double px[5] = {1, x, x * x, x * x * x, x * x * x * x};
        double py[5] = {1, y, y * y, y * y * y, y * y * y * y};
        double pz[5] = {1, z, z * z, z * z * z, z * z * z * z};
        for (int m = 0; m < kNMom; ++m) acc[m] += q * px[c_mom.e[m][0]] * py[c_mom.e[m][1]] * pz[c_mom.e[m][2]];
    }
    for (int m = 0; m < kNMom; ++m) {
        sh[threadIdx.x] = acc[m];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[int64_t(blockIdx.x) * kNMom + m] = sh[0];
        __syncthreads();
    }
}

__global__ void moments_reduce_kernel(int nb, const double* __restrict__ part, double h3, double* __restrict__ mom) {
    const int m = threadIdx.x;
    if (m >= kNMom) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[int64_t(b) * kNMom + m];
    mom[m] = h3 * s;
}

__device__ inline int mom_index(int a, int b, int c) {
    // position of (a, b, c) in the n-major, a-descending, b-descending order
    const int n = a + b + c;
    int k = 0;
    for (int m = 0; m < n; ++m) k += (m + 1) * (m + 2) / 2;
    // within order n: a from n down to 0, for each a, b from n - a down to 0
    for (int aa = n; aa > a; --aa) k += n - aa + 1;
    return k + (n - a - b);
}

__device__ inline double mom(const double* M, int a, int b, int c) { return M[mom_index(a, b, c)]; }

// sum over |alpha| = n of n! / alpha! x^alpha f(alpha)
template <class F>
__device__ inline double contract(int n, double x, double y, double z, F f) {
    const double fact[5] = {1, 1, 2, 6, 24};
    double px[5] = {1, x, x * x, x * x * x, x * x * x * x};
    double py[5] = {1, y, y * y, y * y * y, y * y * y * y};
    double pz[5] = {1, z, z * z, z * z * z, z * z * z * z};
    double s = 0.0;
    for (int a = n; a >= 0; --a)
        for (int b = n - a; b >= 0; --b) {
            const int c = n - a - b;
            s += fact[n] / (fact[a] * fact[b] * fact[c]) * px[a] * py[b] * pz[c] * f(a, b, c);
        }
    return s;
}

__global__ void ghost_values_kernel(int64_t n_ghost, const int32_t* __restrict__ gijk, double h,
                                    const double* __restrict__ M, double* __restrict__ vg) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n_ghost) return;
    const double x = gijk[3 * g] * h, y = gijk[3 * g + 1] * h, z = gijk[3 * g + 2] * h;
    const double r2 = x * x + y * y + z * z;
    const double r = sqrt(r2);
    auto plain = [&](int a, int b, int c) { return mom(M, a, b, c); };
    auto tr1 = [&](int a, int b, int c) { return mom(M, a + 2, b, c) + mom(M, a, b + 2, c) + mom(M, a, b, c + 2); };
    const double T0 = mom(M, 0, 0, 0);
    const double T1 = contract(1, x, y, z, plain);
    const double T2 = contract(2, x, y, z, plain);
    const double T3 = contract(3, x, y, z, plain);
    const double T4 = contract(4, x, y, z, plain);
    const double S0 = tr1(0, 0, 0);
    const double S1 = contract(1, x, y, z, tr1);
    const double S2 = contract(2, x, y, z, tr1);
    const double Q0 = mom(M, 4, 0, 0) + mom(M, 0, 4, 0) + mom(M, 0, 0, 4) +
                      2.0 * (mom(M, 2, 2, 0) + mom(M, 2, 0, 2) + mom(M, 0, 2, 2));
    const double ir = 1.0 / r, ir2 = ir * ir;
    double v = T0 * ir;
    v += T1 * ir * ir2;
    v += (3.0 * T2 - r2 * S0) * 0.5 * ir * ir2 * ir2;
    v += (5.0 * T3 - 3.0 * r2 * S1) * 0.5 * ir * ir2 * ir2 * ir2;
    v += (35.0 * T4 - 30.0 * r2 * S2 + 3.0 * r2 * r2 * Q0) * 0.125 * ir * ir2 * ir2 * ir2 * ir2;
    vg[g] = v;
}

// b[row] = 4 pi rho[row] + sum_{ghosts g of row} (c_|k| / h^2) V(g); 0 on padding
__global__ void poisson_rhs_kernel(int64_t n_rows, const uint8_t* __restrict__ inside, const double* __restrict__ rho,
                                   const int32_t* __restrict__ goff, const int32_t* __restrict__ gk,
                                   const double* __restrict__ vg, const double* __restrict__ ck, double* __restrict__ b) {
    const int64_t row = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (row >= n_rows) return;
    if (!inside[row]) {
        b[row] = 0.0;
        return;
    }
    double s = 4.0 * kPi * rho[row];
    for (int g = goff[row]; g < goff[row + 1]; ++g) s += ck[gk[g]] * vg[g];
    b[row] = s;
}

// v = a x + b y + c z (any of y, z may be null)
__global__ void axpbypcz_kernel(int64_t n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                                double c, const double* __restrict__ z, double* __restrict__ v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = a * x[i];
    if (y) s += b * y[i];
    if (z) s += c * z[i];
    v[i] = s;
}

// sum rho (a - b)^2  (per-block partials, deterministic)
__global__ void __launch_bounds__(256) wdiff2_kernel(int64_t n, const double* __restrict__ w, const double* __restrict__ a,
                                                     const double* __restrict__ b, const double* __restrict__ c,
                                                     const double* __restrict__ d, double* __restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const double dv = (a[i] + b[i]) - (c[i] + d[i]);
        acc += w[i] * dv * dv;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) sum_kernel(int n, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// superposition of Gaussian atoms: rho = sum_a Z_a (alpha_a / pi)^(3/2) exp(-alpha_a r^2)
__global__ void __launch_bounds__(256) sad_kernel(int64_t n_rows, const int32_t* __restrict__ ijk4, double h, int n_atoms,
                                                  const double4* __restrict__ atoms, const double* __restrict__ alpha,
                                                  double* __restrict__ rho) {
    __shared__ double4 sa[256];
    __shared__ double sal[256];
    const int64_t row = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool live = row < n_rows && ijk4[4 * row + 3] != 0;
    double x = 0, y = 0, z = 0;
    if (live) {
        x = ijk4[4 * row] * h;
        y = ijk4[4 * row + 1] * h;
        z = ijk4[4 * row + 2] * h;
    }
    double s = 0.0;
    for (int base = 0; base < n_atoms; base += 256) {
        __syncthreads();
        if (base + threadIdx.x < n_atoms) {
            sa[threadIdx.x] = atoms[base + threadIdx.x];
            sal[threadIdx.x] = alpha[base + threadIdx.x];
        }
        __syncthreads();
        const int cnt = min(256, n_atoms - base);
        if (live)
            for (int t = 0; t < cnt; ++t) {
                const double dx = x - sa[t].x, dy = y - sa[t].y, dz = z - sa[t].z;
                const double al = sal[t];
                const double e = al * (dx * dx + dy * dy + dz * dz);
                if (e < 745.0) s += sa[t].w * pow(al / kPi, 1.5) * exp(-e);
            }
    }
    if (row < n_rows) rho[row] = live ? s : 0.0;
}

__global__ void __launch_bounds__(256) sum_partial_kernel(int64_t n, const double* __restrict__ x,
                                                          double* __restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        acc += x[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void clamp_kernel(int64_t n, double* __restrict__ v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n && !(v[i] > 0.0)) v[i] = 0.0;
}

__global__ void scale_kernel(int64_t n, double a, double* __restrict__ v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) v[i] *= a;
}

static unsigned nblk(int64_t n) { return unsigned((n + 255) / 256); }

static double sum_host(chf_ctx* ctx, int nparts, hipStream_t s) {
    double* out = reinterpret_cast<double*>(ctx->info.p);
    sum_kernel<<<1, 256, 0, s>>>(nparts, ctx->red.as<double>(), out);
    LAUNCH_CHECK();
    double h = 0;
    HIP_CHECK(hipMemcpyAsync(&h, out, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    return h;
}

// ---------------------------------------------------------------------------
// exterior stencil points of the Poisson problem (host build, first use)
// ---------------------------------------------------------------------------
static void build_ghosts(chf_ham* H, hipStream_t s) {
    if (H->n_ghost >= 0) return;
    const HostGrid& g = H->grid;
    std::vector<int32_t> off(size_t(g.n_rows) + 1, 0), kk, ijk;
    std::vector<std::vector<int32_t>> per_row_k(0);
    // rows in ascending order; ghosts of a row in neighbour-column order
    std::vector<int64_t> rank_rows(g.row_of_rank);
    std::vector<int32_t> cnt(size_t(g.n_rows), 0);
    std::vector<std::pair<int64_t, std::array<int32_t, 4>>> items;
    for (int64_t p = 0; p < g.n; ++p) {
        const int i = g.ijk[size_t(3 * p)], j = g.ijk[size_t(3 * p + 1)], k = g.ijk[size_t(3 * p + 2)];
        const int64_t row = g.row_of_rank[size_t(p)];
        for (int axis = 0; axis < 3; ++axis)
            for (int st = -kHalf; st <= kHalf; ++st) {
                if (st == 0) continue;
                const int a = i + (axis == 0 ? st : 0), b = j + (axis == 1 ? st : 0), c = k + (axis == 2 ? st : 0);
                if (g.inside(a, b, c)) continue;
                items.push_back({row, {std::abs(st), a, b, c}});
            }
    }
    std::stable_sort(items.begin(), items.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    kk.reserve(items.size());
    ijk.reserve(items.size() * 3);
    for (auto& it : items) {
        off[size_t(it.first) + 1]++;
        kk.push_back(it.second[0]);
        ijk.push_back(it.second[1]);
        ijk.push_back(it.second[2]);
        ijk.push_back(it.second[3]);
    }
    for (int64_t r = 0; r < g.n_rows; ++r) off[size_t(r) + 1] += off[size_t(r)];
    upload(H->ghost_owner, off, s);
    upload(H->ghost_k, kk, s);
    upload(H->ghost_ijk, ijk, s);
    H->n_ghost = int64_t(kk.size());
    HIP_CHECK(hipStreamSynchronize(s));
}

// Hartree potential into vh (warm start from its contents); returns CG iterations.
int hartree_solve(chf_ham* H, chf_ctx* ctx, const double* rho, double* vh, double rtol, int max_iter, hipStream_t s) {
    build_ghosts(H, s);
    const int64_t n = H->grid.n_rows;
    // workspace: b, r, p, Ap (n each) + ghost values + moments
    const size_t need = size_t(n) * 4 * sizeof(double) + size_t(std::max<int64_t>(1, H->n_ghost)) * sizeof(double) + 4096;
    ctx->vec.ensure(need);
    double* b = ctx->vec.as<double>();
    double* r = b + n;
    double* pv = r + n;
    double* ap = pv + n;
    double* vg = ap + n;
    double* M = vg + std::max<int64_t>(1, H->n_ghost);
    double* ck = M + 64;
    ctx->red.ensure(size_t(1024) * kNMom * sizeof(double));
    const double h = H->h;
    // moments
    const int mb = int(std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256)));
    moments_kernel<<<mb, 256, 0, s>>>(n, H->row_ijk4.as<int32_t>(), h, rho, ctx->red.as<double>());
    LAUNCH_CHECK();
    moments_reduce_kernel<<<1, 64, 0, s>>>(mb, ctx->red.as<double>(), h * h * h, M);
    LAUNCH_CHECK();
    if (H->n_ghost > 0) {
        ghost_values_kernel<<<nblk(H->n_ghost), 256, 0, s>>>(H->n_ghost, H->ghost_ijk.as<int32_t>(), h, M, vg);
        LAUNCH_CHECK();
    }
    // c_k / h^2 for |k| = 1..6 (index by |k|): Laplacian weights = -2 coef
    double ckh[8] = {0};
    for (int k = 1; k <= kHalf; ++k) ckh[k] = -2.0 * H->coef[k];
    HIP_CHECK(hipMemcpyAsync(ck, ckh, sizeof(ckh), hipMemcpyHostToDevice, s));
    poisson_rhs_kernel<<<nblk(n), 256, 0, s>>>(n, H->row_inside.as<uint8_t>(), rho, H->ghost_owner.as<int32_t>(),
                                              H->ghost_k.as<int32_t>(), vg, ck, b);
    LAUNCH_CHECK();
    // A v = -L v = 2 (-1/2 L) v on the inside points (padding stays zero)
    auto apply_a = [&](const double* x, double* y) { hx_step<double>(H, x, 1, y, 1, nullptr, 0, 1, 2.0, 0.0, 0.0, s, 0, true); };
    const double bn = std::sqrt(dot_host<double>(ctx, n, b, 1, b, 1, s));
    apply_a(vh, ap);
    axpbypcz_kernel<<<nblk(n), 256, 0, s>>>(n, 1.0, b, -1.0, ap, 0.0, nullptr, r);
    LAUNCH_CHECK();
    HIP_CHECK(hipMemcpyAsync(pv, r, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
    double rr = dot_host<double>(ctx, n, r, 1, r, 1, s);
    int it = 0;
    while (std::sqrt(rr) > rtol * bn && it < max_iter) {
        apply_a(pv, ap);
        const double alpha = rr / dot_host<double>(ctx, n, pv, 1, ap, 1, s);
        axpbypcz_kernel<<<nblk(n), 256, 0, s>>>(n, 1.0, vh, alpha, pv, 0.0, nullptr, vh);
        axpbypcz_kernel<<<nblk(n), 256, 0, s>>>(n, 1.0, r, -alpha, ap, 0.0, nullptr, r);
        LAUNCH_CHECK();
        const double rr_new = dot_host<double>(ctx, n, r, 1, r, 1, s);
        axpbypcz_kernel<<<nblk(n), 256, 0, s>>>(n, 1.0, r, rr_new / rr, pv, 0.0, nullptr, pv);
        LAUNCH_CHECK();
        rr = rr_new;
        ++it;
    }
    if (!std::isfinite(rr)) fail(CHF_ENONFINITE, "chf_hartree: non-finite residual");
    if (std::sqrt(rr) > rtol * bn) fail(CHF_ENOTCONV, "chf_hartree: CG did not reach %g in %d iterations", rtol, max_iter);
    return it;
}

template <class T>
void density_t(chf_ham* H, const T* X, int64_t ldx, int n_occ, double* rho, hipStream_t s) {
    const int64_t n = H->grid.n_rows;
    const double h = H->h;
    density_kernel<T><<<unsigned((n + 3) / 4), 256, 0, s>>>(n, X, ldx, n_occ, 2.0 / (h * h * h), rho);
    LAUNCH_CHECK();
}

void lda_t(int64_t n, const double* rho, double* exc, double* vxc, hipStream_t s) {
    lda_kernel<<<nblk(n), 256, 0, s>>>(n, rho, exc, vxc);
    LAUNCH_CHECK();
}

}  // namespace chf

// ---------------------------------------------------------------------------
// SCF state
// ---------------------------------------------------------------------------
struct chf_scf {
    chf_ham* H = nullptr;
    chf_ctx* ctx = nullptr;
    chf_scf_params prm{};
    int64_t n = 0;
    int step = 0;
    bool have_bounds = false;
    double a = 0, a0 = 0;
    double e_ion = 0;
    chf::DevBuf fields;          // rho_in, vh, vh_out, vxc_in, exc_in, vxc_out, rho_out, veff, v_lanczos
    chf::DevBuf hist;            // Anderson history: x_j and f_j, mix_history each
    int n_hist = 0;
    std::vector<double> eig;
    double* f(int i) { return fields.as<double>() + int64_t(i) * n; }
    double* hx(int j) { return hist.as<double>() + int64_t(j) * n; }                   // x history
    double* hf(int j) { return hist.as<double>() + int64_t(prm.mix_history + j) * n; } // f history
};

namespace chf {

enum { F_RHO = 0, F_VH, F_VHO, F_VXC, F_EXC, F_VXCO, F_RHOO, F_VEFF, F_VL, F_F, F_TMP, F_COUNT };

__global__ void anderson_dot_kernel(int64_t n, int m, const double* __restrict__ x, const double* __restrict__ f,
                                    const double* __restrict__ hf, int64_t hstride, double* __restrict__ part) {
    // partial sums of dF_j . dF_k (j <= k) and dF_j . f, dF_j = f - f_j
    __shared__ double sh[256];
    const int nterm = m * (m + 1) / 2 + m;
    for (int term = 0; term < nterm; ++term) {
        int j, k;
        bool with_f = term >= m * (m + 1) / 2;
        if (with_f) {
            j = term - m * (m + 1) / 2;
            k = -1;
        } else {
            int t = term;
            j = 0;
            while (t >= m - j) {
                t -= m - j;
                ++j;
            }
            k = j + t;
        }
        double acc = 0.0;
        for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
            const double fi = f[i];
            const double dj = fi - hf[j * hstride + i];
            const double dk = with_f ? fi : fi - hf[k * hstride + i];
            acc += dj * dk;
        }
        sh[threadIdx.x] = acc;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[int64_t(term) * gridDim.x + blockIdx.x] = sh[0];
        __syncthreads();
    }
}

__global__ void anderson_reduce_kernel(int nterm, int nb, const double* __restrict__ part, double* __restrict__ out) {
    const int term = blockIdx.x;
    __shared__ double sh[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) acc += part[int64_t(term) * nb + b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[term] = sh[0];
}

// x_next = (x - sum g_j (x - x_j)) + beta (f - sum g_j (f - f_j)); padding rows keep 0
__global__ void anderson_mix_kernel(int64_t n, int m, const double* __restrict__ g, double beta, const double* __restrict__ x,
                                    const double* __restrict__ f, const double* __restrict__ hx,
                                    const double* __restrict__ hf, int64_t hstride, double* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double xb = x[i], fb = f[i];
    for (int j = 0; j < m; ++j) {
        xb -= g[j] * (x[i] - hx[j * hstride + i]);
        fb -= g[j] * (f[i] - hf[j * hstride + i]);
    }
    out[i] = xb + beta * fb;
}

// small dense solve A g = r (Gaussian elimination with partial pivoting)
static void solve_small(std::vector<double> A, std::vector<double> r, int m, std::vector<double>& g) {
    for (int c = 0; c < m; ++c) {
        int piv = c;
        for (int i = c + 1; i < m; ++i)
            if (std::fabs(A[i * m + c]) > std::fabs(A[piv * m + c])) piv = i;
        if (piv != c) {
            for (int k = 0; k < m; ++k) std::swap(A[c * m + k], A[piv * m + k]);
            std::swap(r[c], r[piv]);
        }
        if (A[c * m + c] == 0.0) fail(CHF_ENONFINITE, "Anderson mixing: singular history");
        for (int i = c + 1; i < m; ++i) {
            const double f = A[i * m + c] / A[c * m + c];
            for (int k = c; k < m; ++k) A[i * m + k] -= f * A[c * m + k];
            r[i] -= f * r[c];
        }
    }
    g.assign(m, 0.0);
    for (int i = m - 1; i >= 0; --i) {
        double s = r[i];
        for (int k = i + 1; k < m; ++k) s -= A[i * m + k] * g[k];
        g[i] = s / A[i * m + i];
    }
}

static void anderson_mix(chf_scf* S, hipStream_t s) {
    const int64_t n = S->n;
    double* x = S->f(F_RHO);
    double* f = S->f(F_F);
    const int m = S->n_hist;
    std::vector<double> gam;
    double* gdev = reinterpret_cast<double*>(S->ctx->info.p);
    if (m > 0) {
        const int nterm = m * (m + 1) / 2 + m;
        const int nb = int(std::min<int64_t>(512, std::max<int64_t>(1, (n + 255) / 256)));
        S->ctx->red.ensure(size_t(nterm) * nb * sizeof(double) + size_t(nterm) * sizeof(double));
        double* part = S->ctx->red.as<double>();
        double* sums = part + int64_t(nterm) * nb;
        // history slots hold (x_j, f_j) oldest first
        std::vector<double> G(m * m), rhs(m);
        anderson_dot_kernel<<<nb, 256, 0, s>>>(n, m, x, f, S->hf(0), n, part);
        LAUNCH_CHECK();
        anderson_reduce_kernel<<<nterm, 256, 0, s>>>(nterm, nb, part, sums);
        LAUNCH_CHECK();
        std::vector<double> hs(nterm);
        HIP_CHECK(hipMemcpyAsync(hs.data(), sums, size_t(nterm) * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        int t = 0;
        for (int j = 0; j < m; ++j)
            for (int k = j; k < m; ++k) {
                G[j * m + k] = G[k * m + j] = hs[t++];
            }
        for (int j = 0; j < m; ++j) rhs[j] = hs[t++];
        solve_small(G, rhs, m, gam);
    }
    if (m > 0) HIP_CHECK(hipMemcpyAsync(gdev, gam.data(), size_t(m) * sizeof(double), hipMemcpyHostToDevice, s));
    double* tmp = S->f(F_TMP);
    anderson_mix_kernel<<<nblk(n), 256, 0, s>>>(n, m, gdev, S->prm.mix_beta, x, f, S->hx(0), S->hf(0), n, tmp);
    LAUNCH_CHECK();
    // push (x, f) into the history (slots kept in insertion order: shift when full)
    if (S->n_hist == S->prm.mix_history) {
        for (int j = 1; j < S->n_hist; ++j) {
            HIP_CHECK(hipMemcpyAsync(S->hx(j - 1), S->hx(j), size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
            HIP_CHECK(hipMemcpyAsync(S->hf(j - 1), S->hf(j), size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        S->n_hist--;
    }
    HIP_CHECK(hipMemcpyAsync(S->hx(S->n_hist), x, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_CHECK(hipMemcpyAsync(S->hf(S->n_hist), f, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
    S->n_hist++;
    HIP_CHECK(hipMemcpyAsync(x, tmp, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
}

static double wsum_host(chf_ctx* ctx, int64_t n, const double* w, const double* a, const double* b, const double* c,
                        const double* d, hipStream_t s) {
    const int nb = int(std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256)));
    ctx->red.ensure(size_t(nb) * sizeof(double));
    wdiff2_kernel<<<nb, 256, 0, s>>>(n, w, a, b, c, d, ctx->red.as<double>());
    LAUNCH_CHECK();
    return sum_host(ctx, nb, s);
}

template <class T>
static void scf_step_t(chf_scf* S, T* X, int64_t ldx, T* W, int64_t ldw, chf_scf_report* rep, double* eig_host) {
    chf_ham* H = S->H;
    chf_ctx* ctx = S->ctx;
    hipStream_t s = H->stream;
    const int64_t n = S->n;
    const double h3 = H->h * H->h * H->h;
    const int n_occ = S->prm.n_electrons / 2;
    const int M = S->prm.nvec;
    S->step++;
    std::memset(rep, 0, sizeof(*rep));
    rep->step = S->step;
    // potentials of rho_in
    int it1 = hartree_solve(H, ctx, S->f(F_RHO), S->f(F_VH), S->prm.cg_rtol, 20000, s);
    lda_t(n, S->f(F_RHO), S->f(F_EXC), S->f(F_VXC), s);
    axpbypcz_kernel<<<nblk(n), 256, 0, s>>>(n, 1.0, H->vloc.as<double>(), 1.0, S->f(F_VH), 1.0, S->f(F_VXC), S->f(F_VEFF));
    LAUNCH_CHECK();
    {
        HIP_CHECK(hipMemsetAsync(H->flag.p, 0, sizeof(int), s));
        launch_cast_veff(H, S->f(F_VEFF), H->veff64.as<double>(), H->veff32.as<float>(), H->flag.as<int>(), s);
        int hbad = 0;
        HIP_CHECK(hipMemcpyAsync(&hbad, H->flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        if (hbad) fail(CHF_ENONFINITE, "scf_step: NaN or Inf in V_eff");
    }
    double bounds[3];
    lanczos_run(H, ctx, S->f(F_VL), S->prm.lanczos_k, bounds, s);
    const double b = bounds[0];
    if (!S->have_bounds) {
        S->a0 = bounds[1];
        S->a = bounds[1] + 0.1 * (b - bounds[1]);
        S->have_bounds = true;
    }
    const int iters = S->step == 1 ? S->prm.first_iters : S->prm.later_iters;
    int fb_total = 0;
    for (int itr = 0; itr < iters; ++itr) {
        rep->bound_a = S->a;
        rep->bound_a0 = S->a0;
        rep->bound_b = b;
        // filter: X <- p_m(H) X, in place over X and W (column blocks of W's width)
        filter_run<T>(H, X, ldx, W, ldw, M, S->prm.degree, S->a, b, S->a0, s, 0);
        int fb = 0;
        orthonormalize_t<T>(ctx, X, ldx, n, M, S->prm.gram_dtype == CHF_F64, &fb, s);
        fb_total += fb;
        rayleigh_ritz_t<T>(H, ctx, X, ldx, M, S->eig.data(), W, ldw, s);
        S->a = S->eig[M - 1];
        S->a0 = S->eig[0];
    }
    rep->chfsi_iters = iters;
    rep->chol_fallbacks = fb_total;
    // output density and its potentials (warm start: V_H of rho_in)
    density_t<T>(H, X, ldx, n_occ, S->f(F_RHOO), s);
    {
        // the output density holds the electron count, h^3 sum rho_out =
        // N_e.  FP64 blocks are orthonormal to rounding (a change of ~1e-14);
        // FP32 blocks only to the accumulation error of their FP32 Gram
        // products, whose systematic part would otherwise add charge and
        // shift the whole potential.
        const int nb = int(std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256)));
        ctx->red.ensure(size_t(nb) * sizeof(double));
        sum_partial_kernel<<<nb, 256, 0, s>>>(n, S->f(F_RHOO), ctx->red.as<double>());
        LAUNCH_CHECK();
        const double q = h3 * sum_host(ctx, nb, s);
        if (!(q > 0)) fail(CHF_ENONFINITE, "scf_step: the output density vanishes");
        scale_kernel<<<nblk(n), 256, 0, s>>>(n, double(S->prm.n_electrons) / q, S->f(F_RHOO));
        LAUNCH_CHECK();
    }
    HIP_CHECK(hipMemcpyAsync(S->f(F_VHO), S->f(F_VH), size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
    int it2 = hartree_solve(H, ctx, S->f(F_RHOO), S->f(F_VHO), S->prm.cg_rtol, 20000, s);
    lda_t(n, S->f(F_RHOO), nullptr, S->f(F_VXCO), s);
    const double sre2 = wsum_host(ctx, n, S->f(F_RHOO), S->f(F_VHO), S->f(F_VXCO), S->f(F_VH), S->f(F_VXC), s);
    rep->sre_ry = 2.0 * std::sqrt(std::max(0.0, h3 * sre2 / S->prm.n_electrons));
    // Harris-Foulkes energy at rho_in
    double band = 0.0;
    for (int i = 0; i < n_occ; ++i) band += S->eig[i];
    band *= 2.0;
    const double rv = dot_host<double>(ctx, n, S->f(F_RHO), 1, S->f(F_VH), 1, s);
    const double rx = dot_host<double>(ctx, n, S->f(F_RHO), 1, S->f(F_VXC), 1, s);
    const double re = dot_host<double>(ctx, n, S->f(F_RHO), 1, S->f(F_EXC), 1, s);
    rep->band_energy = band;
    rep->energy = band - h3 * (rv + rx) + 0.5 * h3 * rv + h3 * re + S->e_ion;
    rep->homo = S->eig[n_occ - 1];
    rep->lumo = n_occ < M ? S->eig[n_occ] : S->eig[M - 1];
    rep->cg_iters = it1 + it2;
    // mix: f = rho_out - rho_in
    axpbypcz_kernel<<<nblk(n), 256, 0, s>>>(n, 1.0, S->f(F_RHOO), -1.0, S->f(F_RHO), 0.0, nullptr, S->f(F_F));
    LAUNCH_CHECK();
    anderson_mix(S, s);
    HIP_CHECK(hipStreamSynchronize(s));
    if (eig_host) std::memcpy(eig_host, S->eig.data(), size_t(M) * sizeof(double));
}

}  // namespace chf

using namespace chf;

template <class F>
static int scf_guard(F&& f) {
    try {
        f();
        return CHF_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return CHF_ENOMEM;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return CHF_EHIP;
    }
}

extern "C" {

int chf_density(chf_ham* H, chf_dtype dtype, const void* X, int64_t ldx, int n_occ, double* rho, void* stream) {
    return scf_guard([&] {
        if (!H || !X || !rho) fail(CHF_EINVAL, "chf_density: null argument");
        if (n_occ < 1 || ldx < n_occ) fail(CHF_EINVAL, "chf_density: need 1 <= n_occ <= ldx");
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (dtype == CHF_F64)
            density_t<double>(H, static_cast<const double*>(X), ldx, n_occ, rho, s);
        else if (dtype == CHF_F32)
            density_t<float>(H, static_cast<const float*>(X), ldx, n_occ, rho, s);
        else
            fail(CHF_EINVAL, "chf_density: bad dtype");
    });
}

int chf_hartree(chf_ham* H, chf_ctx* ctx, const double* rho, double* vh, double rtol, int max_iter, int* iters,
                void* stream) {
    return scf_guard([&] {
        if (!H || !ctx || !rho || !vh) fail(CHF_EINVAL, "chf_hartree: null argument");
        if (!(rtol > 0) || max_iter < 1) fail(CHF_EINVAL, "chf_hartree: need rtol > 0 and max_iter >= 1");
        if (!(H->dtypes & 2)) fail(CHF_EINVAL, "chf_hartree: handle not built for FP64");
        const int it = hartree_solve(H, ctx, rho, vh, rtol, max_iter, static_cast<hipStream_t>(stream));
        if (iters) *iters = it;
    });
}

int chf_lda(chf_ham* H, const double* rho, double* exc, double* vxc, void* stream) {
    return scf_guard([&] {
        if (!H || !rho || !vxc) fail(CHF_EINVAL, "chf_lda: null argument");
        lda_t(H->grid.n_rows, rho, exc, vxc, static_cast<hipStream_t>(stream));
    });
}

int chf_sad_density(chf_ham* H, const chf_atoms* atoms, double alpha_si, double alpha_h, int n_electrons, double* rho,
                    void* stream) {
    return scf_guard([&] {
        if (!H || !atoms || !rho) fail(CHF_EINVAL, "chf_sad_density: null argument");
        if (!(alpha_si > 0 && alpha_h > 0) || n_electrons < 1) fail(CHF_EINVAL, "chf_sad_density: bad parameters");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int na = atoms->n_atoms;
        std::vector<double> at(size_t(std::max(1, na)) * 4, 0.0), al(size_t(std::max(1, na)), 1.0);
        for (int a = 0; a < na; ++a) {
            for (int d = 0; d < 3; ++d) at[size_t(4 * a + d)] = atoms->pos_host[3 * a + d];
            const bool si = atoms->species_host[a] == 0;
            at[size_t(4 * a + 3)] = si ? 4.0 : 1.0;
            al[size_t(a)] = si ? alpha_si : alpha_h;
        }
        DevBuf dat, dal, part, out;
        upload(dat, at, s);
        upload(dal, al, s);
        const int64_t n = H->grid.n_rows;
        sad_kernel<<<nblk(n), 256, 0, s>>>(n, H->row_ijk4.as<int32_t>(), H->h, na, dat.as<double4>(), dal.as<double>(), rho);
        LAUNCH_CHECK();
        const int nb = int(std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256)));
        part.alloc(size_t(nb) * sizeof(double));
        out.alloc(64);
        sum_partial_kernel<<<nb, 256, 0, s>>>(n, rho, part.as<double>());
        LAUNCH_CHECK();
        sum_kernel<<<1, 256, 0, s>>>(nb, part.as<double>(), out.as<double>());
        LAUNCH_CHECK();
        double tot = 0;
        HIP_CHECK(hipMemcpyAsync(&tot, out.p, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        const double h3 = H->h * H->h * H->h;
        if (!(tot > 0)) fail(CHF_ENONFINITE, "chf_sad_density: zero density");
        scale_kernel<<<nblk(n), 256, 0, s>>>(n, n_electrons / (h3 * tot), rho);
        LAUNCH_CHECK();
        HIP_CHECK(hipStreamSynchronize(s));
    });
}

int chf_density_fix(chf_ham* H, double* rho, int n_electrons, void* stream) {
    return scf_guard([&] {
        if (!H || !rho || n_electrons < 1) fail(CHF_EINVAL, "chf_density_fix: bad argument");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int64_t n = H->grid.n_rows;
        clamp_kernel<<<nblk(n), 256, 0, s>>>(n, rho);
        LAUNCH_CHECK();
        const int nbk = int(std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256)));
        DevBuf part, out;
        part.alloc(size_t(nbk) * sizeof(double));
        out.alloc(64);
        sum_partial_kernel<<<nbk, 256, 0, s>>>(n, rho, part.as<double>());
        sum_kernel<<<1, 256, 0, s>>>(nbk, part.as<double>(), out.as<double>());
        LAUNCH_CHECK();
        double tot = 0;
        HIP_CHECK(hipMemcpyAsync(&tot, out.p, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        const double h3 = H->h * H->h * H->h;
        if (!(tot > 0)) fail(CHF_ENONFINITE, "chf_density_fix: density vanishes");
        scale_kernel<<<nblk(n), 256, 0, s>>>(n, n_electrons / (h3 * tot), rho);
        LAUNCH_CHECK();
        HIP_CHECK(hipStreamSynchronize(s));
    });
}

int chf_ion_energy(const chf_atoms* atoms, const chf_pp* pp, double* out) {
    return scf_guard([&] {
        if (!atoms || !pp || !out) fail(CHF_EINVAL, "chf_ion_energy: null argument");
        double e = 0.0;
        for (int a = 0; a < atoms->n_atoms; ++a) {
            const double za = atoms->species_host[a] == 0 ? pp->z_si : pp->z_h;
            const double* pa = atoms->pos_host + 3 * a;
            for (int b = a + 1; b < atoms->n_atoms; ++b) {
                const double zb = atoms->species_host[b] == 0 ? pp->z_si : pp->z_h;
                const double* pb = atoms->pos_host + 3 * b;
                const double dx = pa[0] - pb[0], dy = pa[1] - pb[1], dz = pa[2] - pb[2];
                const double d = std::sqrt(dx * dx + dy * dy + dz * dz);
                if (!(d > 0)) fail(CHF_EINVAL, "chf_ion_energy: coincident atoms");
                e += za * zb / d;
            }
        }
        *out = e;
    });
}

int chf_scf_create(chf_ham* H, chf_ctx* ctx, const chf_scf_params* prm, const double* rho0, const double* v_lanczos,
                   chf_scf** out) {
    return scf_guard([&] {
        if (!H || !ctx || !prm || !rho0 || !v_lanczos || !out) fail(CHF_EINVAL, "chf_scf_create: null argument");
        *out = nullptr;
        if (prm->n_electrons < 2 || prm->n_electrons % 2) fail(CHF_EINVAL, "chf_scf_create: need an even electron count");
        if (prm->nvec <= prm->n_electrons / 2) fail(CHF_EINVAL, "chf_scf_create: nvec must exceed the occupied count");
        if (int64_t(prm->nvec) > H->grid.n)
            fail(CHF_EINVAL, "chf_scf_create: nvec exceeds the grid points (no orthonormal block of that width)");
        if (prm->degree < 1 || prm->first_iters < 1 || prm->later_iters < 1) fail(CHF_EINVAL, "chf_scf_create: bad schedule");
        if (prm->lanczos_k < 2 || prm->lanczos_k > 64) fail(CHF_EINVAL, "chf_scf_create: lanczos_k in [2, 64]");
        if (prm->filter_dtype != CHF_F32 && prm->filter_dtype != CHF_F64) fail(CHF_EINVAL, "chf_scf_create: bad filter dtype");
        if (prm->gram_dtype != CHF_F32 && prm->gram_dtype != CHF_F64) fail(CHF_EINVAL, "chf_scf_create: bad Gram dtype");
        if (prm->filter_dtype == CHF_F64 && prm->gram_dtype != CHF_F64)
            fail(CHF_EINVAL, "chf_scf_create: an FP64 filter needs an FP64 Gram");
        if (prm->mix_history < 0 || prm->mix_history > 32 || !(prm->mix_beta > 0)) fail(CHF_EINVAL, "chf_scf_create: bad mixing");
        if (!(prm->cg_rtol > 0)) fail(CHF_EINVAL, "chf_scf_create: bad CG tolerance");
        if (!(H->dtypes & 2)) fail(CHF_EINVAL, "chf_scf_create: handle must be built with FP64");
        if (!(H->dtypes & (prm->filter_dtype == CHF_F64 ? 2 : 1))) fail(CHF_EINVAL, "chf_scf_create: handle lacks filter dtype");
        auto S = std::make_unique<chf_scf>();
        S->H = H;
        S->ctx = ctx;
        S->prm = *prm;
        S->n = H->grid.n_rows;
        S->e_ion = prm->e_ion;
        S->eig.assign(size_t(prm->nvec), 0.0);
        S->fields.alloc(size_t(S->n) * F_COUNT * sizeof(double));
        HIP_CHECK(hipMemsetAsync(S->fields.p, 0, size_t(S->n) * F_COUNT * sizeof(double), H->stream));
        if (prm->mix_history > 0) S->hist.alloc(size_t(S->n) * 2 * prm->mix_history * sizeof(double));
        HIP_CHECK(hipMemcpyAsync(S->f(F_RHO), rho0, size_t(S->n) * sizeof(double), hipMemcpyDeviceToDevice, H->stream));
        HIP_CHECK(hipMemcpyAsync(S->f(F_VL), v_lanczos, size_t(S->n) * sizeof(double), hipMemcpyDeviceToDevice, H->stream));
        HIP_CHECK(hipStreamSynchronize(H->stream));
        *out = S.release();
    });
}

int chf_scf_destroy(chf_scf* S) {
    if (S) {
        (void)hipDeviceSynchronize();
        delete S;
    }
    return CHF_OK;
}

int scf_step(chf_scf* S, void* X, int64_t ldx, void* W, int64_t ldw, chf_scf_report* rep, double* eig_host) {
    return scf_guard([&] {
        if (!S || !X || !W || !rep) fail(CHF_EINVAL, "scf_step: null argument");
        if (ldx < S->prm.nvec || ldw < 1) fail(CHF_EINVAL, "scf_step: need ldx >= nvec and ldw >= 1");
        check_disjoint(S->H, S->prm.filter_dtype, X, ldx, W, ldw, "scf_step: X and work");
        if (S->prm.filter_dtype == CHF_F64)
            scf_step_t<double>(S, static_cast<double*>(X), ldx, static_cast<double*>(W), ldw, rep, eig_host);
        else
            scf_step_t<float>(S, static_cast<float*>(X), ldx, static_cast<float*>(W), ldw, rep, eig_host);
    });
}

int chf_scf_get_fields(chf_scf* S, double* rho_in, double* vh) {
    return scf_guard([&] {
        if (!S) fail(CHF_EINVAL, "chf_scf_get_fields: null state");
        hipStream_t s = S->H->stream;
        if (rho_in) HIP_CHECK(hipMemcpyAsync(rho_in, S->f(F_RHO), size_t(S->n) * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (vh) HIP_CHECK(hipMemcpyAsync(vh, S->f(F_VH), size_t(S->n) * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIP_CHECK(hipStreamSynchronize(s));
    });
}

// Checkpoint layout (doubles): a header of kCkptHeader values {version,
// step, have_bounds, a, a0, n_hist, n_rows, mix_history}, then rho_in,
// V_H, the n_hist past densities and the n_hist past residuals ([n_rows]
// each, oldest first).
static constexpr int64_t kCkptHeader = 8;
static constexpr double kCkptVersion = 1.0;

int chf_scf_state_size(const chf_scf* S, int64_t* n_doubles) {
    return scf_guard([&] {
        if (!S || !n_doubles) fail(CHF_EINVAL, "chf_scf_state_size: null argument");
        *n_doubles = kCkptHeader + int64_t(2 + 2 * S->n_hist) * S->n;
    });
}

int chf_scf_save(chf_scf* S, double* state_host) {
    return scf_guard([&] {
        if (!S || !state_host) fail(CHF_EINVAL, "chf_scf_save: null argument");
        hipStream_t s = S->H->stream;
        const double hdr[kCkptHeader] = {kCkptVersion, double(S->step), S->have_bounds ? 1.0 : 0.0, S->a, S->a0,
                                         double(S->n_hist), double(S->n), double(S->prm.mix_history)};
        std::memcpy(state_host, hdr, sizeof(hdr));
        const size_t nb = size_t(S->n) * sizeof(double);
        double* out = state_host + kCkptHeader;
        HIP_CHECK(hipMemcpyAsync(out, S->f(F_RHO), nb, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipMemcpyAsync(out + S->n, S->f(F_VH), nb, hipMemcpyDeviceToHost, s));
        for (int j = 0; j < S->n_hist; ++j) {
            HIP_CHECK(hipMemcpyAsync(out + (2 + j) * S->n, S->hx(j), nb, hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipMemcpyAsync(out + (2 + S->n_hist + j) * S->n, S->hf(j), nb, hipMemcpyDeviceToHost, s));
        }
        HIP_CHECK(hipStreamSynchronize(s));
    });
}

int chf_scf_load(chf_scf* S, const double* state_host, int64_t n_doubles) {
    return scf_guard([&] {
        if (!S || !state_host) fail(CHF_EINVAL, "chf_scf_load: null argument");
        if (n_doubles < kCkptHeader) fail(CHF_EINVAL, "chf_scf_load: state too short");
        const double* h = state_host;
        if (h[0] != kCkptVersion) fail(CHF_EINVAL, "chf_scf_load: unknown state version");
        if (int64_t(h[6]) != S->n || int(h[7]) != S->prm.mix_history)
            fail(CHF_EINVAL, "chf_scf_load: state from a different grid or mixing history");
        const int n_hist = int(h[5]);
        if (n_hist < 0 || n_hist > S->prm.mix_history || !(h[1] >= 0))
            fail(CHF_EINVAL, "chf_scf_load: corrupt state header");
        if (n_doubles != kCkptHeader + int64_t(2 + 2 * n_hist) * S->n) fail(CHF_EINVAL, "chf_scf_load: state size mismatch");
        hipStream_t s = S->H->stream;
        const size_t nb = size_t(S->n) * sizeof(double);
        const double* in = state_host + kCkptHeader;
        HIP_CHECK(hipMemcpyAsync(S->f(F_RHO), in, nb, hipMemcpyHostToDevice, s));
        HIP_CHECK(hipMemcpyAsync(S->f(F_VH), in + S->n, nb, hipMemcpyHostToDevice, s));
        for (int j = 0; j < n_hist; ++j) {
            HIP_CHECK(hipMemcpyAsync(S->hx(j), in + (2 + j) * S->n, nb, hipMemcpyHostToDevice, s));
            HIP_CHECK(hipMemcpyAsync(S->hf(j), in + (2 + n_hist + j) * S->n, nb, hipMemcpyHostToDevice, s));
        }
        HIP_CHECK(hipStreamSynchronize(s));
        S->step = int(h[1]);
        S->have_bounds = h[2] != 0.0;
        S->a = h[3];
        S->a0 = h[4];
        S->n_hist = n_hist;
    });
}

}  // extern "C"
