// Hamiltonian application and the Chebyshev filter on gfx950.
//
// Paper: ChFSI's efficiency rests on sparse H-times-wavefunction products;
// the grid points are stored along blockwise Hilbert space-filling curves so
// that these products touch memory with good locality.  H = -1/2 L (12th-
// order FD stencil) + V_eff + sum_a |beta_a> h_l <beta_a| (KB form).
//
// Kernels
//  * vloc_kernel      V_loc on every row (FP64, all atoms, erf screening).
//  * kb_gather        C[a][lm][v] = h^3 sum_q beta_alm(q) X(q, v) per projector atom.
//  * hx_generic       per-row neighbour-table stencil + V + KB scatter, with
//                     the Chebyshev three-term update fused into the store:
//                     Y = alpha (H X - c X) - beta Z  (Z may alias Y).
//  * hx_tiled         the same operator on the Hilbert-blocked layout: one
//                     workgroup per (8^3 block, 32-float / 16-double vector
//                     chunk), z-march with a 13-deep register window per
//                     column, x/y halos staged in LDS (double-buffered).
#include <cmath>

#include "internal.hpp"
#include "kernels.hpp"

namespace chf {

// ---------------------------------------------------------------------------
// local potential
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) vloc_kernel(int64_t n_rows, const int32_t* __restrict__ row_ijk4, double h,
                                                   int n_atoms, const double4* __restrict__ atoms,
                                                   const double* __restrict__ width, double* __restrict__ vloc) {
    __shared__ double4 sa[256];
    __shared__ double sw[256];
    const int64_t row = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool live = row < n_rows && row_ijk4[4 * row + 3] != 0;
    double x = 0, y = 0, z = 0;
    if (live) {
        x = double(row_ijk4[4 * row + 0]) * h;
        y = double(row_ijk4[4 * row + 1]) * h;
        z = double(row_ijk4[4 * row + 2]) * h;
    }
    double v = 0.0;
    const double two_over_sqrt_pi = 1.1283791670955126;
    for (int base = 0; base < n_atoms; base += 256) {
        __syncthreads();
        if (base + threadIdx.x < n_atoms) {
            sa[threadIdx.x] = atoms[base + threadIdx.x];
            sw[threadIdx.x] = width[base + threadIdx.x];
        }
        __syncthreads();
        const int cnt = min(256, n_atoms - base);
        if (live) {
            for (int t = 0; t < cnt; ++t) {
                const double4 a = sa[t];
                const double dx = x - a.x, dy = y - a.y, dz = z - a.z;
                const double d = sqrt(dx * dx + dy * dy + dz * dz);
                const double w = sw[t];
                double term;
                if (d < 1e-8)
                    term = a.w * two_over_sqrt_pi / w;
                else if (d > 6.0 * w)   // erf(x) rounds to exactly 1 in FP64 for x > 5.93
                    term = a.w / d;
                else
                    term = a.w * erf(d / w) / d;
                v -= term;
            }
        }
    }
    if (row < n_rows) vloc[row] = live ? v : 0.0;
}

void launch_vloc(chf_ham* H, const double4* atoms, const double* width, int n_atoms, hipStream_t s) {
    const int64_t n = H->grid.n_rows;
    vloc_kernel<<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, s>>>(n, H->row_ijk4.as<int32_t>(), H->h, n_atoms,
                                                                      atoms, width, H->vloc.as<double>());
    LAUNCH_CHECK();
}

__global__ void cast_veff_kernel(int64_t n, const double* __restrict__ src, const uint8_t* __restrict__ inside,
                                 double* __restrict__ d64, float* __restrict__ d32, int* __restrict__ bad) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = inside[i] ? src[i] : 0.0;
    if (!isfinite(v)) {
        atomicOr(bad, 1);
        return;
    }
    if (d64) d64[i] = v;
    if (d32) d32[i] = float(v);
}

void launch_cast_veff(chf_ham* H, const double* src, double* d64, float* d32, int* bad_dev, hipStream_t s) {
    const int64_t n = H->grid.n_rows;
    cast_veff_kernel<<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, s>>>(n, src, H->row_inside.as<uint8_t>(),
                                                                          d64, d32, bad_dev);
    LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// KB gather: C[a][lm][v] = sum_j (h^3 beta_alm(row_j)) X[row_j][v]
// 256 threads = 64 vector lanes x 4 slices of the support list; the slices
// are summed in fixed order (deterministic).
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) kb_gather_kernel(const int64_t* __restrict__ sup_off,
                                                        const int32_t* __restrict__ sup_row,
                                                        const T* __restrict__ sup_beta, const T* __restrict__ X,
                                                        int64_t ldx, int nvec, T* __restrict__ C) {
    __shared__ T part[4][4][64];
    const int a = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int slice = threadIdx.x >> 6;
    const int v = blockIdx.y * 64 + lane;
    const int64_t j0 = sup_off[a], j1 = sup_off[a + 1];
    T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    if (v < nvec) {
        for (int64_t j = j0 + slice; j < j1; j += 4) {
            const T x = X[int64_t(sup_row[j]) * ldx + v];
            const T* b = sup_beta + 4 * j;
            s0 += b[0] * x;
            s1 += b[1] * x;
            s2 += b[2] * x;
            s3 += b[3] * x;
        }
    }
    part[slice][0][lane] = s0;
    part[slice][1][lane] = s1;
    part[slice][2][lane] = s2;
    part[slice][3][lane] = s3;
    __syncthreads();
    if (slice == 0 && v < nvec) {
        for (int lm = 0; lm < 4; ++lm) {
            const T t = ((part[0][lm][lane] + part[1][lm][lane]) + part[2][lm][lane]) + part[3][lm][lane];
            C[(int64_t(a) * 4 + lm) * nvec + v] = t;
        }
    }
}

template <class T>
void launch_kb_gather(chf_ham* H, const T* X, int64_t ldx, int nvec, T* C, hipStream_t s) {
    if (H->proj.n_proj == 0) return;
    const T* beta = std::is_same<T, double>::value ? H->sup_beta64.as<T>() : H->sup_beta32.as<T>();
    dim3 grid(unsigned(H->proj.n_proj), unsigned((nvec + 63) / 64));
    kb_gather_kernel<T><<<grid, dim3(256), 0, s>>>(H->sup_off.as<int64_t>(), H->sup_row.as<int32_t>(), beta, X, ldx,
                                                   nvec, C);
    LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// generic neighbour-table H X with fused recurrence epilogue
// ---------------------------------------------------------------------------
template <class T>
struct StepCoef {
    T c[7];        // -1/2 c_k / h^2 (c[0] already multiplied by 3: three axes)
    T alpha, shift, beta;
};

template <class T>
__global__ void __launch_bounds__(256) hx_generic_kernel(int64_t n_rows, int nvec, int nvc,
                                                         const int32_t* __restrict__ nbr,
                                                         const uint8_t* __restrict__ inside,
                                                         const T* __restrict__ veff,
                                                         const int64_t* __restrict__ ent_off,
                                                         const int32_t* __restrict__ ent_atom,
                                                         const T* __restrict__ ent_beta, const T* __restrict__ C,
                                                         const T* __restrict__ X, int64_t ldx, T* Y, int64_t ldy,
                                                         const T* Z, int64_t ldz, StepCoef<T> k) {
    const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t row = gid / nvc;
    const int vc = int(gid - row * nvc);
    if (row >= n_rows) return;
    constexpr int VPT = 4;
    const int v0 = vc * VPT;
    if (!inside[row]) {
        for (int e = 0; e < VPT; ++e)
            if (v0 + e < nvec) Y[row * ldy + v0 + e] = T(0);
        return;
    }
    T xc[VPT], acc[VPT];
    const T* xr = X + row * ldx;
    for (int e = 0; e < VPT; ++e) {
        xc[e] = (v0 + e < nvec) ? xr[v0 + e] : T(0);
        acc[e] = k.c[0] * xc[e];
    }
    const int32_t* nb = nbr + row * kNbr;
#pragma unroll
    for (int col = 0; col < kNbr; ++col) {
        const int32_t r = nb[col];
        const int kk = (col % 12) < 6 ? 6 - (col % 12) : (col % 12) - 5;
        if (r >= 0) {
            const T* q = X + int64_t(r) * ldx;
            for (int e = 0; e < VPT; ++e)
                if (v0 + e < nvec) acc[e] += k.c[kk] * q[v0 + e];
        }
    }
    const T vr = veff[row];
    for (int e = 0; e < VPT; ++e) acc[e] += vr * xc[e];
    for (int64_t en = ent_off[row]; en < ent_off[row + 1]; ++en) {
        const int64_t a = ent_atom[en];
        const T* b = ent_beta + 4 * en;
        const T* ca = C + a * 4 * nvec;
        for (int e = 0; e < VPT; ++e)
            if (v0 + e < nvec)
                acc[e] += b[0] * ca[v0 + e] + b[1] * ca[nvec + v0 + e] + b[2] * ca[2 * nvec + v0 + e] +
                          b[3] * ca[3 * nvec + v0 + e];
    }
    for (int e = 0; e < VPT; ++e) {
        if (v0 + e >= nvec) continue;
        T y = k.alpha * (acc[e] - k.shift * xc[e]);
        if (Z) y -= k.beta * Z[row * ldz + v0 + e];
        Y[row * ldy + v0 + e] = y;
    }
}

template <class T>
StepCoef<T> make_coef(const chf_ham* H, double alpha, double shift, double beta) {
    StepCoef<T> k;
    k.c[0] = T(3.0 * H->coef[0]);
    for (int i = 1; i < 7; ++i) k.c[i] = T(H->coef[i]);
    k.alpha = T(alpha);
    k.shift = T(shift);
    k.beta = T(beta);
    return k;
}

template <class T>
static const T* veff_of(const chf_ham* H) {
    return std::is_same<T, double>::value ? H->veff64.as<T>() : H->veff32.as<T>();
}
template <class T>
static const T* ent_beta_of(const chf_ham* H) {
    return std::is_same<T, double>::value ? H->ent_beta64.as<T>() : H->ent_beta32.as<T>();
}

template <class T>
void launch_hx_generic(chf_ham* H, const T* X, int64_t ldx, T* Y, int64_t ldy, const T* Z, int64_t ldz, int nvec,
                       const T* C, double alpha, double shift, double beta, hipStream_t s) {
    const int nvc = (nvec + 3) / 4;
    const int64_t total = H->grid.n_rows * nvc;
    hx_generic_kernel<T><<<dim3(unsigned((total + 255) / 256)), dim3(256), 0, s>>>(
        H->grid.n_rows, nvec, nvc, H->nbr_rows.as<int32_t>(), H->row_inside.as<uint8_t>(), veff_of<T>(H),
        H->ent_off.as<int64_t>(), H->ent_atom.as<int32_t>(), ent_beta_of<T>(H), C, X, ldx, Y, ldy, Z, ldz,
        make_coef<T>(H, alpha, shift, beta));
    LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Hilbert-blocked tiled H X
//
// Workgroup: 512 threads = 64 columns (x, y) of one 8^3 block x 8 "quads"
// of 16 bytes (4 floats or 2 doubles) -> a 128-byte vector chunk per row
// (32 FP32 or 16 FP64 vectors).  Each thread keeps X(x, y, z-6 .. z+6) of
// its column and quad in registers and marches z = 0..7; the x/y neighbours
// of plane z (the plane plus its 6-deep halos from the -x/+x/-y/+y
// neighbour blocks) are staged in LDS, double-buffered so that one barrier
// per plane suffices.  The KB scatter reads the per-row entry lists and the
// coefficients C of the step; the Chebyshev update is fused into the store.
// Rows outside the sphere are stored as zero; on input they must hold zero
// (the layout contract), so they enter the stencil as the zero boundary.
//
// LDS plane layout (rows of 128 B): a 20 x 8 strip for x in [-6, 14) and
// y in [0, 8) (160 rows) followed by two 8 x 6 strips for y in [-6, 0) and
// [8, 14) (48 rows each): 256 rows = 32 KB per plane, 64 KB double-buffered.
// ---------------------------------------------------------------------------
template <class T>
struct Quad;
template <>
struct Quad<float> {
    using V = float4;
    static constexpr int N = 4;
};
template <>
struct Quad<double> {
    using V = double2;
    static constexpr int N = 2;
};

template <class V>
__device__ inline V vzero();
template <>
__device__ inline float4 vzero<float4>() { return make_float4(0.f, 0.f, 0.f, 0.f); }
template <>
__device__ inline double2 vzero<double2>() { return make_double2(0.0, 0.0); }

__device__ inline float4 vfma(float s, float4 a, float4 c) {
    return make_float4(fmaf(s, a.x, c.x), fmaf(s, a.y, c.y), fmaf(s, a.z, c.z), fmaf(s, a.w, c.w));
}
__device__ inline double2 vfma(double s, double2 a, double2 c) { return make_double2(fma(s, a.x, c.x), fma(s, a.y, c.y)); }
__device__ inline float4 vadd(float4 a, float4 b) { return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }
__device__ inline double2 vadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline float4 vscale(float s, float4 a) { return make_float4(s * a.x, s * a.y, s * a.z, s * a.w); }
__device__ inline double2 vscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

__device__ inline int lds_row(int x, int y) {
    // x in [-6, 14), y in [-6, 14), not both outside [0, 8)
    if (y >= 0 && y < 8) return (x + 6) + 20 * y;
    if (y < 0) return 160 + x + 8 * (y + 6);
    return 208 + x + 8 * (y - 8);
}

template <class T>
__global__ void __launch_bounds__(512) hx_tiled_kernel(int64_t n_blocks, int n_chunks, const int32_t* __restrict__ bnb,
                                                       const uint64_t* __restrict__ bmask, const T* __restrict__ veff,
                                                       const int64_t* __restrict__ ent_off,
                                                       const int32_t* __restrict__ ent_atom,
                                                       const T* __restrict__ ent_beta, const T* __restrict__ C,
                                                       int nvec, const T* __restrict__ X, int64_t ldx, T* Y,
                                                       int64_t ldy, const T* Z, int64_t ldz, StepCoef<T> k) {
    using V = typename Quad<T>::V;
    constexpr int QN = Quad<T>::N;       // elements per quad
    constexpr int CH = 8 * QN;           // vectors per chunk
    __shared__ V plane[2][256][8];

    // XCD-aware tile order: workgroup ids are dealt round-robin to the 8
    // XCDs; give each XCD a contiguous run of the (chunk-major, Hilbert-
    // ordered) tile sequence so that neighbouring blocks share its L2.
    const int64_t ntiles = n_blocks * n_chunks;
    const int64_t wg = blockIdx.x;
    const int64_t per_xcd = (ntiles + 7) / 8;
    const int64_t xcd = wg % 8, idx = wg / 8;
    const int64_t tile = xcd * per_xcd + idx;
    if (tile >= ntiles) return;
    const int chunk = int(tile / n_blocks);
    const int64_t blk = tile - int64_t(chunk) * n_blocks;

    const int t = threadIdx.x;
    const int q = t & 7;                 // quad within the chunk
    const int col = t >> 3;              // column 0..63
    const int cx = col & 7, cy = col >> 3;
    const int vbase = chunk * CH + q * QN;
    const bool vok = vbase < nvec;       // nvec is a multiple of QN (host-checked)

    int32_t nbs[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) nbs[f] = bnb[6 * blk + f];
    uint64_t mymask[8];
#pragma unroll
    for (int w = 0; w < 8; ++w) mymask[w] = bmask[8 * blk + w];

    auto inside_local = [&](int l) -> bool { return (mymask[l >> 6] >> (l & 63)) & 1; };
    auto load_row = [&](int64_t row) -> V {
        return vok ? *reinterpret_cast<const V*>(X + row * ldx + vbase) : vzero<V>();
    };

    // register window: w[i] = X(cx, cy, z - 6 + i), i = 0..19; rows are
    // loaded one plane ahead of use so that about 14 are live at a time.
    V w[20];
    const int64_t base = blk * kBlockPts;
    auto load_plane = [&](int zz) -> V {
        if (zz < 0) {
            if (nbs[4] >= 0) return load_row(int64_t(nbs[4]) * kBlockPts + cx + 8 * cy + 64 * (zz + 8));
            return vzero<V>();
        }
        if (zz >= 8) {
            if (nbs[5] >= 0) return load_row(int64_t(nbs[5]) * kBlockPts + cx + 8 * cy + 64 * (zz - 8));
            return vzero<V>();
        }
        return load_row(base + cx + 8 * cy + 64 * zz);
    };
#pragma unroll
    for (int i = 0; i < 14; ++i) w[i] = load_plane(i - 6);
    // Rows outside the sphere hold zeros in every buffer (layout contract),
    // so halo rows need no mask: a missing neighbour block reads as zero.

    // halo loader for plane z into buffer b: 192 halo rows x 8 quads = 1536
    // quad loads, 3 per thread.
    auto load_halo = [&](int z, int b) {
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int hidx = t + 512 * u;          // 0..1535
            const int hq = hidx & 7;
            const int hr = hidx >> 3;              // 0..191
            int side = hr / 48;                    // 0:-x 1:+x 2:-y 3:+y
            int rem = hr % 48;
            int lx, ly, nbx, x, y;
            if (side < 2) {
                // 6 columns x 8 rows of y
                const int c6 = rem % 6;
                ly = rem / 6;
                lx = side == 0 ? 2 + c6 : c6;      // local x in the neighbour block
                x = side == 0 ? c6 - 6 : 8 + c6;   // x in this block's frame
                y = ly;
            } else {
                const int r6 = rem / 8;
                lx = rem % 8;
                ly = side == 2 ? 2 + r6 : r6;
                x = lx;
                y = side == 2 ? r6 - 6 : 8 + r6;
            }
            nbx = nbs[side];
            V val = vzero<V>();
            if (nbx >= 0) {
                const int64_t r = int64_t(nbx) * kBlockPts + lx + 8 * ly + 64 * z;
                if (chunk * CH + hq * QN < nvec)
                    val = *reinterpret_cast<const V*>(X + r * ldx + chunk * CH + hq * QN);
            }
            plane[b][lds_row(x, y)][hq] = val;
        }
    };

    load_halo(0, 0);
    plane[0][lds_row(cx, cy)][q] = w[6];
    __syncthreads();

    const T* vr = veff + base;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const int b = z & 1;
        if (z < 7) {
            load_halo(z + 1, b ^ 1);
            plane[b ^ 1][lds_row(cx, cy)][q] = w[z + 7];
        }
        if (z < 6) w[z + 14] = load_plane(z + 8);
        const int l = cx + 8 * cy + 64 * z;
        const int64_t row = base + l;
        V acc = vscale(k.c[0], w[z + 6]);
#pragma unroll
        for (int s = 1; s <= 6; ++s) {
            V sum = vadd(w[z + 6 - s], w[z + 6 + s]);
            sum = vadd(sum, plane[b][lds_row(cx - s, cy)][q]);
            sum = vadd(sum, plane[b][lds_row(cx + s, cy)][q]);
            sum = vadd(sum, plane[b][lds_row(cx, cy - s)][q]);
            sum = vadd(sum, plane[b][lds_row(cx, cy + s)][q]);
            acc = vfma(k.c[s], sum, acc);
        }
        if (vok && !inside_local(l)) {
            *reinterpret_cast<V*>(Y + row * ldy + vbase) = vzero<V>();
        } else if (vok) {
            const V xc = w[z + 6];
            acc = vfma(vr[l], xc, acc);
            const int64_t e0 = ent_off[row], e1 = ent_off[row + 1];
            for (int64_t en = e0; en < e1; ++en) {
                const int64_t a = ent_atom[en];
                const T* bb = ent_beta + 4 * en;
                const T* ca = C + a * 4 * int64_t(nvec) + vbase;
                acc = vfma(bb[0], *reinterpret_cast<const V*>(ca), acc);
                acc = vfma(bb[1], *reinterpret_cast<const V*>(ca + nvec), acc);
                acc = vfma(bb[2], *reinterpret_cast<const V*>(ca + 2 * nvec), acc);
                acc = vfma(bb[3], *reinterpret_cast<const V*>(ca + 3 * nvec), acc);
            }
            V y = vscale(k.alpha, vfma(-k.shift, xc, acc));
            if (Z) y = vfma(-k.beta, *reinterpret_cast<const V*>(Z + row * ldz + vbase), y);
            *reinterpret_cast<V*>(Y + row * ldy + vbase) = y;
        }
        __syncthreads();
    }
}

template <class T>
void launch_hx_tiled(chf_ham* H, const T* X, int64_t ldx, T* Y, int64_t ldy, const T* Z, int64_t ldz, int nvec,
                     const T* C, double alpha, double shift, double beta, hipStream_t s) {
    constexpr int CH = 8 * Quad<T>::N;
    const int n_chunks = (nvec + CH - 1) / CH;
    const int64_t nt = H->grid.n_blocks * n_chunks;
    const int64_t nwg = ((nt + 7) / 8) * 8;
    hx_tiled_kernel<T><<<dim3(unsigned(nwg)), dim3(512), 0, s>>>(
        H->grid.n_blocks, n_chunks, H->block_nbr.as<int32_t>(), H->block_mask.as<uint64_t>(), veff_of<T>(H),
        H->ent_off.as<int64_t>(), H->ent_atom.as<int32_t>(), ent_beta_of<T>(H), C, nvec, X, ldx, Y, ldy, Z, ldz,
        make_coef<T>(H, alpha, shift, beta));
    LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <class T>
bool tiled_ok(const chf_ham* H, const void* X, int64_t ldx, const void* Y, int64_t ldy, const void* Z, int64_t ldz,
              int nvec) {
    constexpr int QN = Quad<T>::N;
    if (H->grid.ordering != CHF_ORDER_HILBERT) return false;
    if (nvec % QN || ldx % QN || ldy % QN || (Z && ldz % QN)) return false;
    const uintptr_t al = 16;
    if (uintptr_t(X) % al || uintptr_t(Y) % al || (Z && uintptr_t(Z) % al)) return false;
    return true;
}

template <class T>
void hx_step(chf_ham* H, const T* X, int64_t ldx, T* Y, int64_t ldy, const T* Z, int64_t ldz, int nvec, double alpha,
             double shift, double beta, hipStream_t s, int force_kernel) {
    H->kb_coef.ensure(size_t(std::max<int64_t>(1, H->proj.n_proj)) * 4 * size_t(nvec) * sizeof(T));
    T* C = H->kb_coef.as<T>();
    launch_kb_gather<T>(H, X, ldx, nvec, C, s);
    const bool tiled = force_kernel != 1 && tiled_ok<T>(H, X, ldx, Y, ldy, Z, ldz, nvec);
    if (tiled) {
        launch_hx_tiled<T>(H, X, ldx, Y, ldy, Z, ldz, nvec, C, alpha, shift, beta, s);
    } else {
        if (!H->has_nbr) fail(CHF_EUNSUPPORTED, "generic H X needs the neighbour table (keep_nbr) for this layout");
        launch_hx_generic<T>(H, X, ldx, Y, ldy, Z, ldz, nvec, C, alpha, shift, beta, s);
    }
}

template void hx_step<float>(chf_ham*, const float*, int64_t, float*, int64_t, const float*, int64_t, int, double,
                             double, double, hipStream_t, int);
template void hx_step<double>(chf_ham*, const double*, int64_t, double*, int64_t, const double*, int64_t, int,
                              double, double, double, hipStream_t, int);
template void launch_kb_gather<float>(chf_ham*, const float*, int64_t, int, float*, hipStream_t);
template void launch_kb_gather<double>(chf_ham*, const double*, int64_t, int, double*, hipStream_t);

}  // namespace chf
