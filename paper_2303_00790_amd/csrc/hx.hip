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
//  * hx_tile          the same operator on the Hilbert-blocked layout: one
//                     workgroup per (8^3 block, 32-float / 16-double vector
//                     chunk), z-march with a 20-deep register window per
//                     column, x/y halos staged in LDS (double-buffered), the
//                     block atoms' KB coefficients staged in LDS and the KB
//                     term applied inside the march.
//  * hx_tiled         the same tile without staging, for blocks touched by
//                     more than kMaxBlockAtoms projector atoms, Laplacian-only
//                     products and Hamiltonians without projectors.
#include <atomic>
#include <cmath>
#include <mutex>
#include <type_traits>

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
// generic neighbour-table H X with fused recurrence epilogue
// ---------------------------------------------------------------------------
template <class T>
struct StepCoef {
    T c[7];        // -1/2 c_k / h^2 (c[0] already multiplied by 3: three axes)
    T alpha, shift, beta;
    // the same step with alpha folded in (tiled kernel):
    //   y = sum_k ac[k] (X(p+k) + X(p-k)) + (d0 + alpha V(p)) X(p) + alpha KB - beta Z
    T ac[7];       // alpha c[k], k >= 1 (ac[0] unused)
    T d0;          // alpha (c[0] - shift)
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
    if (veff) {
        const T vr = veff[row];
        for (int e = 0; e < VPT; ++e) acc[e] += vr * xc[e];
    }
    if (ent_off)
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
    k.ac[0] = T(0);
    for (int i = 1; i < 7; ++i) k.ac[i] = T(alpha * H->coef[i]);
    k.d0 = T(alpha * (3.0 * H->coef[0] - shift));
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
                       const T* C, double alpha, double shift, double beta, hipStream_t s, bool lap_only) {
    const int nvc = (nvec + 3) / 4;
    const int64_t total = H->grid.n_rows * nvc;
    hx_generic_kernel<T><<<dim3(unsigned((total + 255) / 256)), dim3(256), 0, s>>>(
        H->grid.n_rows, nvec, nvc, H->nbr_rows.as<int32_t>(), H->row_inside.as<uint8_t>(),
        lap_only ? nullptr : veff_of<T>(H), lap_only ? nullptr : H->ent_off.as<int64_t>(), H->ent_atom.as<int32_t>(),
        ent_beta_of<T>(H), C, X, ldx, Y, ldy, Z, ldz,
        make_coef<T>(H, alpha, shift, beta));
    LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Hilbert-blocked tiled H X (hx_tiled_kernel below)
//
// One workgroup per tile = one 8^3 block x one 128-byte vector chunk (32 FP32
// or 16 FP64 vectors): 1024 threads = 64 columns (x, y) x 16 lanes of 8
// bytes.  Each thread keeps X(x, y, z-6 .. z+13) of its column and lane in
// registers and marches z = 0..7; the x/y neighbours of plane z (the plane
// plus its 6-deep halos from the -x/+x/-y/+y neighbour blocks) are staged in
// LDS as a 20 x 20 square, double-buffered so that one barrier per plane
// suffices.  The KB term of each row is applied in the march from the
// block's staged coefficients; the Chebyshev update is fused into the store.
// Rows outside the sphere are stored as zero; on input they must hold zero
// (the layout contract), so they enter the stencil as the zero boundary.
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

// ---------------------------------------------------------------------------
// KB gather: C[a][lm][v] = sum_j (h^3 beta_alm(row_j)) X[row_j][v]
// One workgroup per (projector atom, 64-quad vector chunk): 4 waves split the
// support list (row j goes to wave j % 4), each lane owns one 16-byte quad of
// vectors, and every lane keeps four independent row loads in flight.  The
// four wave partials are summed in fixed order (deterministic).
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) kb_gather_kernel(const int64_t* __restrict__ sup_off,
                                                        const int32_t* __restrict__ sup_row,
                                                        const T* __restrict__ sup_beta, const T* __restrict__ X,
                                                        int64_t ldx, int nvec, T* __restrict__ C, int n_proj) {
    using V = typename Quad<T>::V;
    constexpr int QN = Quad<T>::N;
    __shared__ V part[4][4][64];
    // XCD-aware order (grid = 8 * per_xcd): consecutive atoms, which share
    // support rows (the device numbers atoms along the Hilbert curve), run on
    // the same XCD and read the shared rows from its L2
    const int per_xcd = int(gridDim.x / 8);
    const int a = int(blockIdx.x % 8) * per_xcd + int(blockIdx.x / 8);
    if (a >= n_proj) return;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int v = (blockIdx.y * 64 + lane) * QN;
    const bool ok = v < nvec;
    const int64_t j0 = sup_off[a], j1 = sup_off[a + 1];
    V s0 = vzero<V>(), s1 = vzero<V>(), s2 = vzero<V>(), s3 = vzero<V>();
    int64_t j = j0 + wave;
    for (; j + 12 < j1; j += 16) {
        V x[4];
        T bt[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t jj = j + 4 * u;
            x[u] = ok ? *reinterpret_cast<const V*>(X + int64_t(sup_row[jj]) * ldx + v) : vzero<V>();
#pragma unroll
            for (int m = 0; m < 4; ++m) bt[u][m] = sup_beta[4 * jj + m];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            s0 = vfma(bt[u][0], x[u], s0);
            s1 = vfma(bt[u][1], x[u], s1);
            s2 = vfma(bt[u][2], x[u], s2);
            s3 = vfma(bt[u][3], x[u], s3);
        }
    }
    for (; j < j1; j += 4) {
        const V x = ok ? *reinterpret_cast<const V*>(X + int64_t(sup_row[j]) * ldx + v) : vzero<V>();
        const T* b = sup_beta + 4 * j;
        s0 = vfma(b[0], x, s0);
        s1 = vfma(b[1], x, s1);
        s2 = vfma(b[2], x, s2);
        s3 = vfma(b[3], x, s3);
    }
    part[wave][0][lane] = s0;
    part[wave][1][lane] = s1;
    part[wave][2][lane] = s2;
    part[wave][3][lane] = s3;
    __syncthreads();
    if (ok) {
        const int lm = wave;   // each wave finishes one channel
        const V t = vadd(vadd(vadd(part[0][lm][lane], part[1][lm][lane]), part[2][lm][lane]), part[3][lm][lane]);
        *reinterpret_cast<V*>(C + (int64_t(a) * 4 + lm) * nvec + v) = t;
    }
}

// scalar variant for blocks whose width or alignment rules out 16-byte quads
template <class T>
__global__ void __launch_bounds__(256) kb_gather_scalar_kernel(const int64_t* __restrict__ sup_off,
                                                               const int32_t* __restrict__ sup_row,
                                                               const T* __restrict__ sup_beta,
                                                               const T* __restrict__ X, int64_t ldx, int nvec,
                                                               T* __restrict__ C) {
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
    if (v < nvec) {
        const int lm = slice;
        C[(int64_t(a) * 4 + lm) * nvec + v] = ((part[0][lm][lane] + part[1][lm][lane]) + part[2][lm][lane]) + part[3][lm][lane];
    }
}

template <class T>
void launch_kb_gather(chf_ham* H, const T* X, int64_t ldx, int nvec, T* C, hipStream_t s) {
    if (H->proj.n_proj == 0) return;
    constexpr int QN = Quad<T>::N;
    const T* beta = std::is_same<T, double>::value ? H->sup_beta64.as<T>() : H->sup_beta32.as<T>();
    if (nvec % QN == 0 && ldx % QN == 0 && uintptr_t(X) % 16 == 0) {
        dim3 grid(unsigned(8 * ((H->proj.n_proj + 7) / 8)), unsigned((nvec / QN + 63) / 64));
        kb_gather_kernel<T><<<grid, dim3(256), 0, s>>>(H->sup_off.as<int64_t>(), H->sup_row.as<int32_t>(), beta, X, ldx,
                                                       nvec, C, int(H->proj.n_proj));
    } else {
        dim3 grid(unsigned(H->proj.n_proj), unsigned((nvec + 63) / 64));
        kb_gather_scalar_kernel<T><<<grid, dim3(256), 0, s>>>(H->sup_off.as<int64_t>(), H->sup_row.as<int32_t>(), beta,
                                                              X, ldx, nvec, C);
    }
    LAUNCH_CHECK();
}

// 8-byte lane values of the tiled kernel: two floats or one double
template <class T>
struct Lane;
template <>
struct Lane<float> {
    using V = float2;
    static constexpr int N = 2;
};
template <>
struct Lane<double> {
    using V = double;
    static constexpr int N = 1;
};
__device__ inline void lzero(float2& v) { v = make_float2(0.f, 0.f); }
__device__ inline void lzero(double& v) { v = 0.0; }
__device__ inline float2 lfma(float s, float2 a, float2 c) { return make_float2(fmaf(s, a.x, c.x), fmaf(s, a.y, c.y)); }
__device__ inline double lfma(double s, double a, double c) { return fma(s, a, c); }
__device__ inline float2 ladd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline double ladd(double a, double b) { return a + b; }
__device__ inline float2 lscale(float s, float2 a) { return make_float2(s * a.x, s * a.y); }
__device__ inline double lscale(double s, double a) { return s * a; }

template <class V>
__device__ inline V lz() {
    V v;
    lzero(v);
    return v;
}

// compile-time loop: f(integral_constant<int, K>) for K = B .. E-1
template <int B, int E, class F>
__device__ inline void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// value of lane K of this lane's 16-lane row (DPP row_newbcast).  All rows
// and banks are written and the source lane is always valid, so no old value
// is needed (mov_dpp leaves it undefined and saves a register clear).
template <int K>
__device__ inline int row_bcast(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0x150 + K, 0xF, 0xF, false);
}
template <int K>
__device__ inline float row_bcast(float v) {
    return __builtin_bit_cast(float, row_bcast<K>(__builtin_bit_cast(int, v)));
}
template <int K>
__device__ inline double row_bcast(double v) {
    const int2 w = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(row_bcast<K>(w.x), row_bcast<K>(w.y)));
}

__device__ inline void load4(const float* p, float* o) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x, o[1] = v.y, o[2] = v.z, o[3] = v.w;
}
__device__ inline void load4(const double* p, double* o) {
    const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
    o[0] = a.x, o[1] = a.y, o[2] = b.x, o[3] = b.y;
}

// raw buffer access (vector memory through a 128-bit resource descriptor)
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, int(bytes), 0x00020000);
}
template <class V>
__device__ inline V bload(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <class V>
__device__ inline void bstore(V v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}

// Unstaged tile kernel: one workgroup per tile (one 8^3 block x one 128-byte
// vector chunk), 1024 threads = 64 columns x 16 lanes; a lane holds 8 bytes
// (2 floats or 1 double) of the chunk.  It serves the blocks the staged tile
// kernel below cannot take (more than kMaxBlockAtoms projector atoms touch
// the block), the Laplacian-only products of the Poisson solver and
// Hamiltonians without projectors: the stencil is applied in a z-march, the
// eight output rows wait in registers, and the KB term is added after the
// march from the coefficients in global memory.
constexpr int kMaxBlockAtoms = 64;
constexpr int kLanes = 16;

template <class T>
__global__ void __launch_bounds__(64 * kLanes) hx_tiled_kernel(int64_t n_blocks, int n_chunks, const int32_t* __restrict__ bnb,
                                                         const uint64_t* __restrict__ bmask, const T* __restrict__ veff,
                                                         const int32_t* __restrict__ ent_off,
                                                         const int32_t* __restrict__ ent_atom,
                                                         const T* __restrict__ ent_beta, const T* __restrict__ C,
                                                         int nvec, const T* __restrict__ X, int64_t ldx, T* Y,
                                                         int64_t ldy, const T* Z, int64_t ldz, StepCoef<T> k) {
    using V = typename Lane<T>::V;
    constexpr int LANES = kLanes;
    constexpr int LN = Lane<T>::N;       // elements per lane
    constexpr int CH = LANES * LN;       // vectors per chunk
    constexpr int LSH = 4;
    constexpr int CPW = 64 / LANES;      // columns per wave
    // LDS plane: the full 20 x 20 square x in [-6, 14), y in [-6, 14) (corners
    // unused) so every neighbour is a constant offset from the centre
    __shared__ V plane[2][400][LANES];

    // XCD-aware tile order: workgroup ids are dealt round-robin to the 8
    // XCDs; give each XCD a contiguous run of the tile sequence (blocks in
    // Hilbert order, the vector chunks of a block adjacent) so that
    // neighbouring blocks share its L2 and the chunks of a block share the
    // block's tables (KB entries, V_eff, masks).
    const int64_t ntiles = n_blocks * n_chunks;
    const int64_t per_xcd = (ntiles + 7) / 8;
    const int64_t tile = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (tile >= ntiles) return;

    const int t = threadIdx.x;
    const int p = t & (LANES - 1);       // lane within the chunk
    const int col = t >> LSH;            // column 0..63
    const int cx = col & 7, cy = col >> 3;
    const int wave = t >> 6;
    const unsigned es = sizeof(T);
    const unsigned blk_bytes = unsigned(kBlockPts) * unsigned(ldx) * es;
    constexpr unsigned kOOB = 0x80000000u;
    const unsigned plane_x = 64u * unsigned(ldx) * es;
    const unsigned plane_z = 64u * unsigned(ldz) * es;
    const unsigned plane_y = 64u * unsigned(ldy) * es;
    const int ctr = (cy + 6) * 20 + (cx + 6);
    auto res_x = [&](int32_t nb) {
        return make_rsrc(nb >= 0 ? X + int64_t(nb) * kBlockPts * ldx : X, nb >= 0 ? blk_bytes : 0u);
    };

    const int64_t blk = tile / n_chunks;
    const int chunk = int(tile - blk * n_chunks);
    int32_t nbs[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) nbs[f] = bnb[6 * blk + f];
    const int vbase = chunk * CH + p * LN;
    const bool vok = vbase < nvec;
    const unsigned off_x = vok ? (unsigned(cx + 8 * cy) * unsigned(ldx) + unsigned(vbase)) * es : kOOB;
    const unsigned off_z = vok ? (unsigned(cx + 8 * cy) * unsigned(ldz) + unsigned(vbase)) * es : kOOB;
    const __amdgpu_buffer_rsrc_t rOwn = res_x(int32_t(blk));
    const __amdgpu_buffer_rsrc_t rZm = res_x(nbs[4]);
    const __amdgpu_buffer_rsrc_t rZp = res_x(nbs[5]);
    const __amdgpu_buffer_rsrc_t rZ =
        make_rsrc(Z ? Z + blk * kBlockPts * ldz : X, Z ? unsigned(kBlockPts) * unsigned(ldz) * es : 0u);
    // Halo slot u of a wave covers CPW consecutive halo rows, all on one side
    // of the block (48 rows per side), so the side is wave-uniform.
    int hrow[3];
    __amdgpu_buffer_rsrc_t rH[3];
    unsigned hoff[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        const int hr0 = CPW * wave + 64 * u;
        const int side = __builtin_amdgcn_readfirstlane(hr0 / 48);
        const int hr = col + 64 * u;
        const int rem = hr - 48 * side;
        int lx, ly, x, y, nb;
        if (side < 2) {
            const int c6 = rem % 6;
            ly = rem / 6;
            lx = side == 0 ? 2 + c6 : c6;
            x = side == 0 ? c6 - 6 : 8 + c6;
            y = ly;
            nb = side == 0 ? nbs[0] : nbs[1];
        } else {
            const int r6 = rem / 8;
            lx = rem % 8;
            ly = side == 2 ? 2 + r6 : r6;
            x = lx;
            y = side == 2 ? r6 - 6 : 8 + r6;
            nb = side == 2 ? nbs[2] : nbs[3];
        }
        hrow[u] = (y + 6) * 20 + (x + 6);
        rH[u] = res_x(__builtin_amdgcn_readfirstlane(nb));
        hoff[u] = vok ? (unsigned(lx + 8 * ly) * unsigned(ldx) + unsigned(vbase)) * es : kOOB;
    }
    auto load_plane = [&](int zz) -> V {
        if (zz < 0) return bload<V>(rZm, off_x + unsigned(zz + 8) * plane_x);
        if (zz >= 8) return bload<V>(rZp, off_x + unsigned(zz - 8) * plane_x);
        return bload<V>(rOwn, off_x + unsigned(zz) * plane_x);
    };
    auto load_halo = [&](int z, V* hv) {
#pragma unroll
        for (int u = 0; u < 3; ++u) hv[u] = bload<V>(rH[u], hoff[u] + unsigned(z) * plane_x);
    };
    auto store_halo = [&](int b, const V* hv) {
#pragma unroll
        for (int u = 0; u < 3; ++u) plane[b][hrow[u]][p] = hv[u];
    };
    auto load_z = [&](int z) -> V { return bload<V>(rZ, off_z + unsigned(z) * plane_z); };

    const int64_t base = blk * kBlockPts;
    const int lrow = cx + 8 * cy;             // this column's row in plane 0
    // the X window of this column, the first two halo planes and Y_{k-1} of
    // plane 0
    V w[20];
#pragma unroll
    for (int i = 0; i < 14; ++i) w[i] = load_plane(i - 6);
    V hv0[3], hv[3];
    load_halo(0, hv0);
    load_halo(1, hv);
    V zcur = load_z(0);
    store_halo(0, hv0);
    plane[0][ctr][p] = w[6];
    __syncthreads();

    const __amdgpu_buffer_rsrc_t rY = make_rsrc(Y + base * ldy, unsigned(kBlockPts) * unsigned(ldy) * es);
    const unsigned off_y = vok ? (unsigned(lrow) * unsigned(ldy) + unsigned(vbase)) * es : kOOB;
    V r[8];
    const T* vr = veff ? veff + base : nullptr;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const int b = z & 1;
        // stage plane z + 1 (its loads were issued one plane ago), then
        // issue the loads for planes further ahead
        if (z < 7) {
            store_halo(b ^ 1, hv);
            plane[b ^ 1][ctr][p] = w[z + 7];
        }
        if (z < 6) load_halo(z + 2, hv);
        V znext = lz<V>();
        if (z < 7) znext = load_z(z + 1);
        if (z < 6) w[z + 14] = load_plane(z + 8);

        // unscaled stencil (c_0 x + sum_s c_s (six neighbours at distance s))
        V acc = lscale(k.c[0], w[z + 6]);
#pragma unroll
        for (int s = 1; s <= 6; ++s) {
            V sum = ladd(w[z + 6 - s], w[z + 6 + s]);
            sum = ladd(sum, plane[b][ctr - s][p]);
            sum = ladd(sum, plane[b][ctr + s][p]);
            sum = ladd(sum, plane[b][ctr - 20 * s][p]);
            sum = ladd(sum, plane[b][ctr + 20 * s][p]);
            acc = lfma(k.c[s], sum, acc);
        }
        const V xc = w[z + 6];
        if (vr) acc = lfma(vr[lrow + 64 * z], xc, acc);
        V y = lscale(k.alpha, lfma(-k.shift, xc, acc));
        if (Z) y = lfma(-k.beta, zcur, y);
        r[z] = y;
        zcur = znext;
        __syncthreads();
    }

    // KB scatter after the march, in rounds so that the entry loads of all
    // eight rows are in flight together
    if (ent_off && vok) {
        int e0[8], e1[8];
        int nmax = 0;
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            const int64_t row = base + lrow + 64 * z;
            e0[z] = ent_off[row];
            e1[z] = ent_off[row + 1];
            nmax = max(nmax, e1[z] - e0[z]);
        }
        for (int j = 0; j < nmax; ++j) {
#pragma unroll
            for (int z = 0; z < 8; ++z) {
                const int en = e0[z] + j;
                if (en < e1[z]) {
                    const T* bb = ent_beta + 4 * int64_t(en);
                    const T* ca = C + int64_t(ent_atom[en]) * 4 * int64_t(nvec) + vbase;
                    V acc = lscale(bb[0], *reinterpret_cast<const V*>(ca));
                    acc = lfma(bb[1], *reinterpret_cast<const V*>(ca + nvec), acc);
                    acc = lfma(bb[2], *reinterpret_cast<const V*>(ca + 2 * nvec), acc);
                    acc = lfma(bb[3], *reinterpret_cast<const V*>(ca + 3 * nvec), acc);
                    r[z] = lfma(k.alpha, acc, r[z]);
                }
            }
        }
    }
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const bool in = (bmask[8 * blk + z] >> lrow) & 1;
        bstore<V>(in ? r[z] : lz<V>(), rY, off_y + unsigned(z) * plane_y);
    }
}

// ---------------------------------------------------------------------------
// Staged tile kernel: the Hilbert-blocked H X + recurrence with the KB term
// applied inside the z-march from coefficients staged in LDS (blocks touched
// by at most kMaxBlockAtoms projector atoms).  Same tile shape as above: one
// workgroup per (8^3 block, 128-byte vector chunk), 1024 threads = 64
// columns x 16 lanes of 8 bytes; a wave holds 4 columns of one row of the
// block's plane, i.e. one aligned quad of 4 consecutive grid rows.
//
// The KB term of row r is sum_e h_l beta_lm(e) C_lm[slot(e)].  Lane i of a
// column holds entry i of its row (LDS byte offset of the slot's staged
// coefficients and h_l beta_lm), loaded two planes ahead; the wave walks the
// entries up to the largest count among its quad's 4 rows (a per-block table
// gives that count per quad and plane, so the loop bound is wave-uniform and
// the loop needs no per-lane tests); lanes past their row's count hold zero
// weights and add exact zeros.  Per pair of entries: one DPP add per entry
// forms the LDS address (broadcast offset + lane base), two 16-byte LDS reads
// fetch the coefficients, and FMAs with a DPP broadcast operand (row_newbcast
// of the 16-lane group) apply them (FP64: one entry at a time, which keeps
// the kernel within 128 registers).  Every DPP sequence starts with s_nop 1,
// and an accumulator is written at most once every four FMAs, so no DPP
// operand is read within two instructions of the VALU write that made it.
// ---------------------------------------------------------------------------
template <int K>
__device__ inline void bcast_add2(int v, int add, int& r0, int& r1) {
    asm("s_nop 1\n\t"
        "v_add_u32_dpp %0, %2, %3 row_newbcast:%4 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_u32_dpp %1, %2, %3 row_newbcast:%5 row_mask:0xf bank_mask:0xf"
        : "=&v"(r0), "=&v"(r1)
        : "v"(v), "v"(add), "n"(K), "n"(K + 1));
}

// a0..a3 += entry K and K+1 of (b0..b3) times the staged coefficients
// ca = {ch0 v0, ch0 v1, ch1 v0, ch1 v1}, cb = {ch2 v0, ch2 v1, ch3 v0, ch3 v1}
template <int K>
__device__ inline void kb_fma2(float& a0, float& a1, float& a2, float& a3, float b0, float b1, float b2, float b3,
                               float4 ca, float4 cb, float4 da, float4 db) {
    asm("s_nop 1\n\t"
        "v_fmac_f32_dpp %0, %4, %8 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %4, %9 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %5, %10 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %5, %11 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %6, %12 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %6, %13 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %7, %14 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %7, %15 row_newbcast:%24 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %4, %16 row_newbcast:%25 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %4, %17 row_newbcast:%25 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %5, %18 row_newbcast:%25 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %5, %19 row_newbcast:%25 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %6, %20 row_newbcast:%25 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %6, %21 row_newbcast:%25 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %7, %22 row_newbcast:%25 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %7, %23 row_newbcast:%25 row_mask:0xf bank_mask:0xf"
        : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3)
        : "v"(b0), "v"(b1), "v"(b2), "v"(b3), "v"(ca.x), "v"(ca.y), "v"(ca.z), "v"(ca.w), "v"(cb.x), "v"(cb.y),
          "v"(cb.z), "v"(cb.w), "v"(da.x), "v"(da.y), "v"(da.z), "v"(da.w), "v"(db.x), "v"(db.y), "v"(db.z),
          "v"(db.w), "n"(K), "n"(K + 1));
}

// FP64, one entry: a0..a3 += entry K of (b0..b3) times ca = {ch0, ch1}, cb = {ch2, ch3}
template <int K>
__device__ inline void kb_fma1(double& a0, double& a1, double& a2, double& a3, double b0, double b1, double b2,
                               double b3, double2 ca, double2 cb) {
    asm("s_nop 1\n\t"
        "v_fmac_f64_dpp %0, %4, %8 row_newbcast:%12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %1, %5, %9 row_newbcast:%12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %2, %6, %10 row_newbcast:%12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f64_dpp %3, %7, %11 row_newbcast:%12 row_mask:0xf bank_mask:0xf"
        : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3)
        : "v"(b0), "v"(b1), "v"(b2), "v"(b3), "v"(ca.x), "v"(ca.y), "v"(cb.x), "v"(cb.y), "n"(K));
}

template <int K>
__device__ inline int bcast_add1(int v, int add) {
    int r;
    asm("s_nop 1\n\t"
        "v_add_u32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
        : "=v"(r)
        : "v"(v), "v"(add), "n"(K));
    return r;
}

template <class T>
struct KbLds;
template <>
struct KbLds<float> {
    using C = float4;   // coefficients of one channel pair for the lane's 2 vectors
};
template <>
struct KbLds<double> {
    using C = double2;  // one channel pair for the lane's vector
};

template <class V>
__device__ inline V bload_s(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, voff, int(soff), 0));
}
// streaming access (non-temporal cache policy): Y_{k-1} is read and Y_{k+1}
// written once per launch, so they should not displace the X rows that
// neighbouring tiles read again as halos
template <class V>
__device__ inline V bload_nt(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, voff, int(soff), 2));
}
template <class V>
__device__ inline void bstore_nt(V v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, int(soff), 2);
}

// LDS of the staged tile kernel: staged KB coefficients first (their
// addresses fit the 16-bit offset field of the LDS instructions), then the
// two x/y planes
constexpr int kCstBytes = kMaxBlockAtoms * 2 * 16 * 2 * 8;      // [slot][pair][lane][2] x 8 B
constexpr int kPlaneBytes = 2 * 400 * 16 * 8;                   // [2][400][lane] x 8 B
constexpr int kSlotBytes = 2 * 16 * 2 * 8;                      // one slot: 512 B

template <class T>
__global__ void __launch_bounds__(1024) hx_tile_kernel(int64_t n_blocks, int n_chunks, const int32_t* __restrict__ bnb,
                                                       const uint64_t* __restrict__ bmask, const T* __restrict__ veff,
                                                       const int32_t* __restrict__ ent_off,
                                                       const int32_t* __restrict__ ent_soff,
                                                       const T* __restrict__ ent_beta,
                                                       const uint64_t* __restrict__ qcnt,
                                                       const int32_t* __restrict__ blk_atom_off,
                                                       const int32_t* __restrict__ blk_atoms, const T* __restrict__ C,
                                                       int nvec, const T* __restrict__ X, int64_t ldx, T* Y,
                                                       int64_t ldy, const T* Z, int64_t ldz, StepCoef<T> k) {
    using V = typename Lane<T>::V;
    using CL = typename KbLds<T>::C;
    constexpr int LANES = 16;
    constexpr int LN = Lane<T>::N;
    constexpr int CH = LANES * LN;
    constexpr int NT = 64 * LANES;
    constexpr int LSH = 4;
    constexpr int CPW = 4;
    __shared__ __align__(16) char lds[kCstBytes + kPlaneBytes];
    V (*plane)[400][LANES] = reinterpret_cast<V (*)[400][LANES]>(lds + kCstBytes);
    V (*cst)[2][LANES][2] = reinterpret_cast<V (*)[2][LANES][2]>(lds);

    // XCD-aware tile order, as in the unstaged kernel: each XCD takes a
    // contiguous run of the tile sequence.  FP32 tiles run block-major (a
    // block's vector chunks adjacent, sharing its tables and staged
    // coefficients in L2); FP64 tiles run chunk-major (each chunk's blocks
    // along the Hilbert curve, so the tiles in flight on an XCD are
    // neighbouring blocks whose halos overlap), which measured faster for
    // the FP64 kernel, whose traffic sits near the copy ceiling.
    const int64_t ntiles = n_blocks * n_chunks;
    const int64_t per_xcd = (ntiles + 7) / 8;
    const int64_t tile = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (tile >= ntiles) return;

    const int t = threadIdx.x;
    const int p = t & (LANES - 1);
    const int col = t >> LSH;
    const int cx = col & 7, cy = col >> 3;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const unsigned es = sizeof(T);
    const unsigned blk_bytes = unsigned(kBlockPts) * unsigned(ldx) * es;
    constexpr unsigned kOOB = 0x80000000u;
    const unsigned plane_x = 64u * unsigned(ldx) * es;
    const unsigned plane_z = 64u * unsigned(ldz) * es;
    const unsigned plane_y = 64u * unsigned(ldy) * es;
    const int ctr = (cy + 6) * 20 + (cx + 6);
    auto res_x = [&](int32_t nb) {
        return make_rsrc(nb >= 0 ? X + int64_t(nb) * kBlockPts * ldx : X, nb >= 0 ? blk_bytes : 0u);
    };

    constexpr bool chunk_major = sizeof(T) == 8;
    const int64_t blk = chunk_major ? tile % n_blocks : tile / n_chunks;
    const int chunk = chunk_major ? int(tile / n_blocks) : int(tile - blk * n_chunks);
    int32_t nbs[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) nbs[f] = bnb[6 * blk + f];
    const int vbase = chunk * CH + p * LN;
    const bool vok = vbase < nvec;
    const unsigned off_x = vok ? (unsigned(cx + 8 * cy) * unsigned(ldx) + unsigned(vbase)) * es : kOOB;
    const unsigned off_z = vok ? (unsigned(cx + 8 * cy) * unsigned(ldz) + unsigned(vbase)) * es : kOOB;
    const __amdgpu_buffer_rsrc_t rOwn = res_x(int32_t(blk));
    const __amdgpu_buffer_rsrc_t rZm = res_x(nbs[4]);
    const __amdgpu_buffer_rsrc_t rZp = res_x(nbs[5]);
    const __amdgpu_buffer_rsrc_t rZ =
        make_rsrc(Z ? Z + blk * kBlockPts * ldz : X, Z ? unsigned(kBlockPts) * unsigned(ldz) * es : 0u);
    // halo slot u of a wave covers CPW consecutive halo rows, all on one side
    int hrow[3];
    __amdgpu_buffer_rsrc_t rH[3];
    unsigned hoff[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        const int hr0 = CPW * wave + 64 * u;
        const int side = __builtin_amdgcn_readfirstlane(hr0 / 48);
        const int hr = col + 64 * u;
        const int rem = hr - 48 * side;
        int lx, ly, x, y, nb;
        if (side < 2) {
            const int c6 = rem % 6;
            ly = rem / 6;
            lx = side == 0 ? 2 + c6 : c6;
            x = side == 0 ? c6 - 6 : 8 + c6;
            y = ly;
            nb = side == 0 ? nbs[0] : nbs[1];
        } else {
            const int r6 = rem / 8;
            lx = rem % 8;
            ly = side == 2 ? 2 + r6 : r6;
            x = lx;
            y = side == 2 ? r6 - 6 : 8 + r6;
            nb = side == 2 ? nbs[2] : nbs[3];
        }
        hrow[u] = (y + 6) * 20 + (x + 6);
        rH[u] = res_x(__builtin_amdgcn_readfirstlane(nb));
        hoff[u] = vok ? (unsigned(lx + 8 * ly) * unsigned(ldx) + unsigned(vbase)) * es : kOOB;
    }
    auto load_plane = [&](int zz) -> V {
        if (zz < 0) return bload_s<V>(rZm, off_x, unsigned(zz + 8) * plane_x);
        if (zz >= 8) return bload_s<V>(rZp, off_x, unsigned(zz - 8) * plane_x);
        return bload_s<V>(rOwn, off_x, unsigned(zz) * plane_x);
    };
    auto load_halo = [&](int z, V* hv) {
#pragma unroll
        for (int u = 0; u < 3; ++u) hv[u] = bload_s<V>(rH[u], hoff[u], unsigned(z) * plane_x);
    };
    auto store_halo = [&](int b, const V* hv) {
#pragma unroll
        for (int u = 0; u < 3; ++u) plane[b][hrow[u]][p] = hv[u];
    };

    const int64_t base = blk * kBlockPts;
    const int lrow = cx + 8 * cy;
    // KB entries of the block: a buffer over its entries, so that lanes past
    // their row's count read zeros (out-of-range buffer loads return 0)
    const int e_blk0 = ent_off[base];
    const int e_cnt = ent_off[base + kBlockPts] - e_blk0;
    const uint64_t qc8 = qcnt[blk * 16 + wave];
    V cstage[4];
    {
        const int a0 = blk_atom_off[blk];
        const int na = min(blk_atom_off[blk + 1] - a0, kMaxBlockAtoms);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = t + NT * u;         // (atom slot, lm, lane)
            const int sl = e >> (LSH + 2), lm = (e >> LSH) & 3, lp = e & (LANES - 1);
            const int vb = chunk * CH + lp * LN;
            if (sl < na && vb < nvec)         // staged with alpha applied
                cstage[u] = lscale(k.alpha, *reinterpret_cast<const V*>(C + (int64_t(blk_atoms[a0 + sl]) * 4 + lm) * nvec + vb));
            else
                cstage[u] = lz<V>();
        }
    }
    const __amdgpu_buffer_rsrc_t rB = make_rsrc(ent_beta + 4 * int64_t(e_blk0), unsigned(e_cnt) * 4u * es);
    const __amdgpu_buffer_rsrc_t rS = make_rsrc(ent_soff + e_blk0, unsigned(e_cnt) * 4u);
    // entries of row z: lane i holds entry i (LDS byte offset of its slot's
    // coefficients and its 4 weights); the row's entry range comes RL planes
    // before the entries, which come PD planes before their use (both 1 for
    // FP64, whose 4 weights take twice the registers)
    constexpr int PD = sizeof(T) == 4 ? 2 : 1;
    constexpr int RL = sizeof(T) == 4 ? 2 : 1;   // lead of the entry ranges over the entries
    int2 e_rng[8];
    int e_soff[8];
    T e_b[8][4];
    // (a dword-aligned 8-byte load: the row's first entry and the next row's)
    auto load_range = [&](int z) { __builtin_memcpy(&e_rng[z], ent_off + base + lrow + 64 * z, sizeof(int2)); };
    auto load_entries = [&](int z) {
        const int en = e_rng[z].x + p;
        const unsigned rel = unsigned(en - e_blk0);
        const bool ok = en < e_rng[z].y;
        e_soff[z] = int(__builtin_amdgcn_raw_buffer_load_b32(rS, ok ? rel * 4u : kOOB, 0, 0));
        if constexpr (sizeof(T) == 4) {
            const float4 b4 = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rB, ok ? rel * 16u : kOOB, 0, 0));
            e_b[z][0] = b4.x, e_b[z][1] = b4.y, e_b[z][2] = b4.z, e_b[z][3] = b4.w;
        } else {
            const unsigned o = ok ? rel * 32u : kOOB;
            const double2 b0 = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rB, o, 0, 0));
            const double2 b1 = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rB, o, 16, 0));
            e_b[z][0] = b0.x, e_b[z][1] = b0.y, e_b[z][2] = b1.x, e_b[z][3] = b1.y;
        }
    };
#pragma unroll
    for (int z = 0; z < PD + RL; ++z) load_range(z);
    // the X window of this column, the first two halo planes, Y_{k-1} and
    // V_eff of plane 0
    // (X planes are loaded WL planes before the stencil first needs them: 2,
    // or 1 for FP64 to stay within 128 registers)
    constexpr int WL = sizeof(T) == 4 ? 2 : 1;
    V w[20];
#pragma unroll
    for (int i = 0; i < 12 + WL; ++i) w[i] = load_plane(i - 6);
    V hv0[3], hv[3];
    load_halo(0, hv0);
    load_halo(1, hv);
    V zcur = bload_nt<V>(rZ, off_z, 0u);      // zero when there is no Z (empty buffer)
    T vcur = veff[base + lrow];
#pragma unroll
    for (int z = 0; z < PD; ++z) load_entries(z);
    store_halo(0, hv0);
    plane[0][ctr][p] = w[6];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = t + NT * u;
        const int sl = e >> (LSH + 2), lm = (e >> LSH) & 3, lp = e & (LANES - 1);
        if (sl < kMaxBlockAtoms) cst[sl][lm >> 1][lp][lm & 1] = cstage[u];
    }
    __syncthreads();

    const __amdgpu_buffer_rsrc_t rY = make_rsrc(Y + base * ldy, unsigned(kBlockPts) * unsigned(ldy) * es);
    const unsigned off_y = vok ? (unsigned(lrow) * unsigned(ldy) + unsigned(vbase)) * es : kOOB;
    const int lane_off = p * 16;           // this lane's 16 bytes within a slot's channel pair
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const int b = z & 1;
        if (z < 7) {
            store_halo(b ^ 1, hv);
            plane[b ^ 1][ctr][p] = w[z + 7];
        }
        // loads, in the order they are needed: next plane's halos, Y_{k-1}
        // and V_eff first, then the entries of plane z + PD, the entry range
        // of plane z + PD + RL and the X plane z + 8
        if (z < 6) load_halo(z + 2, hv);
        V znext = lz<V>();
        T vnext = T(0);
        if (z < 7) {
            znext = bload_nt<V>(rZ, off_z, unsigned(z + 1) * plane_z);
            vnext = veff[base + lrow + 64 * (z + 1)];
        }
        if (z + PD < 8) load_entries(z + PD);
        if (z + PD + RL < 8) load_range(z + PD + RL);
        if (z + 6 + WL < 14) w[z + 12 + WL] = load_plane(z + 6 + WL);

        // alpha-scaled off-diagonal stencil; the diagonal is added last
        V acc = lz<V>();
#pragma unroll
        for (int s = 1; s <= 6; ++s) {
            V sum = ladd(w[z + 6 - s], w[z + 6 + s]);
            sum = ladd(sum, plane[b][ctr - s][p]);
            sum = ladd(sum, plane[b][ctr + s][p]);
            sum = ladd(sum, plane[b][ctr - 20 * s][p]);
            sum = ladd(sum, plane[b][ctr + 20 * s][p]);
            acc = s == 1 ? lscale(k.ac[1], sum) : lfma(k.ac[s], sum, acc);
        }
        const V xc = w[z + 6];
        {
            // KB term of row z: entries in pairs up to the quad's largest count
            const int qc = int((qc8 >> (8 * z)) & 0xffu);
            T a[4];
            if constexpr (sizeof(T) == 4) {
                a[0] = acc.x, a[1] = acc.y, a[2] = 0.f, a[3] = 0.f;
            } else {
                a[0] = acc, a[1] = 0.0, a[2] = 0.0, a[3] = 0.0;
            }
            if constexpr (sizeof(T) == 4) {
                static_for<0, 8>([&](auto gc) {
                    constexpr int kk = 2 * decltype(gc)::value;
                    if (kk < qc) {
                        int ad0, ad1;
                        bcast_add2<kk>(e_soff[z], lane_off, ad0, ad1);
                        const CL ca = *reinterpret_cast<const CL*>(lds + ad0);
                        const CL cb = *reinterpret_cast<const CL*>(lds + ad0 + 256);
                        const CL da = *reinterpret_cast<const CL*>(lds + ad1);
                        const CL db = *reinterpret_cast<const CL*>(lds + ad1 + 256);
                        kb_fma2<kk>(a[0], a[1], a[2], a[3], e_b[z][0], e_b[z][1], e_b[z][2], e_b[z][3], ca, cb, da,
                                    db);
                    }
                });
            } else {
                static_for<0, 16>([&](auto kc) {
                    constexpr int kk = decltype(kc)::value;
                    if (kk < qc) {
                        const int ad = bcast_add1<kk>(e_soff[z], lane_off);
                        const CL ca = *reinterpret_cast<const CL*>(lds + ad);
                        const CL cb = *reinterpret_cast<const CL*>(lds + ad + 256);
                        kb_fma1<kk>(a[0], a[1], a[2], a[3], e_b[z][0], e_b[z][1], e_b[z][2], e_b[z][3], ca, cb);
                    }
                });
            }
            if (qc > 16) {                    // rows with more than 16 entries: the rest from memory
                int2 rng;
                __builtin_memcpy(&rng, ent_off + base + lrow + 64 * z, sizeof(int2));
                for (int en = rng.x + 16; en < rng.y; ++en) {
                    const T* bb = ent_beta + 4 * int64_t(en);
                    const char* cs = lds + ent_soff[en] + lane_off;
                    const CL c01 = *reinterpret_cast<const CL*>(cs);
                    const CL c23 = *reinterpret_cast<const CL*>(cs + 256);
                    if constexpr (sizeof(T) == 4) {
                        a[0] = fmaf(bb[0], c01.x, a[0]);
                        a[1] = fmaf(bb[0], c01.y, a[1]);
                        a[2] = fmaf(bb[1], c01.z, a[2]);
                        a[3] = fmaf(bb[1], c01.w, a[3]);
                        a[0] = fmaf(bb[2], c23.x, a[0]);
                        a[1] = fmaf(bb[2], c23.y, a[1]);
                        a[2] = fmaf(bb[3], c23.z, a[2]);
                        a[3] = fmaf(bb[3], c23.w, a[3]);
                    } else {
                        a[0] = fma(bb[0], c01.x, a[0]);
                        a[1] = fma(bb[1], c01.y, a[1]);
                        a[2] = fma(bb[2], c23.x, a[2]);
                        a[3] = fma(bb[3], c23.y, a[3]);
                    }
                }
            }
            if constexpr (sizeof(T) == 4)
                acc = make_float2(a[0] + a[2], a[1] + a[3]);
            else
                acc = (a[0] + a[1]) + (a[2] + a[3]);
        }
        const T dg = T(fma(k.alpha, vcur, k.d0));
        V y = lfma(dg, xc, acc);
        y = lfma(-k.beta, zcur, y);            // beta = 0 when there is no Z
        // rows outside the sphere are stored as zero: the wave's quad is rows
        // 4 wave .. 4 wave + 3 of the plane, 16 lanes each
        const uint64_t m4 = (bmask[8 * blk + z] >> (4 * wave)) & 0xfu;
        const uint64_t spread = (m4 & 1u) | ((m4 & 2u) << 15) | ((m4 & 4u) << 30) | ((m4 & 8u) << 45);
        const bool in = __builtin_amdgcn_inverse_ballot_w64(spread * 0xffffu);
        bstore_nt<V>(in ? y : lz<V>(), rY, off_y, unsigned(z) * plane_y);
        zcur = znext;
        vcur = vnext;
        __syncthreads();
    }
}

template <class T>
void launch_hx_tiled(chf_ham* H, const T* X, int64_t ldx, T* Y, int64_t ldy, const T* Z, int64_t ldz, int nvec,
                     const T* C, double alpha, double shift, double beta, hipStream_t s, bool lap_only) {
    constexpr int CH = kLanes * Lane<T>::N;
    const int n_chunks = (nvec + CH - 1) / CH;
    const int64_t nt = H->grid.n_blocks * int64_t(n_chunks);
    const dim3 grid(unsigned(((nt + 7) / 8) * 8)), block(64 * kLanes);
    const bool kb = !lap_only && H->proj.n_proj > 0;
    const bool stage = kb && H->proj.max_block_atoms <= kMaxBlockAtoms;
    const int32_t* eo = kb ? H->ent_off32.as<int32_t>() : nullptr;
    const StepCoef<T> coef = make_coef<T>(H, alpha, shift, beta);
    const T* veff = lap_only ? nullptr : veff_of<T>(H);
    if (stage)
        hx_tile_kernel<T><<<grid, block, 0, s>>>(H->grid.n_blocks, n_chunks, H->block_nbr.as<int32_t>(),
                                                H->block_mask.as<uint64_t>(), veff, eo, H->ent_soff.as<int32_t>(),
                                                ent_beta_of<T>(H), H->quad_count.as<uint64_t>(),
                                                H->blk_atom_off.as<int32_t>(), H->blk_atoms.as<int32_t>(), C, nvec, X,
                                                ldx, Y, ldy, Z, ldz, coef);
    else
        hx_tiled_kernel<T><<<grid, block, 0, s>>>(H->grid.n_blocks, n_chunks, H->block_nbr.as<int32_t>(),
                                                 H->block_mask.as<uint64_t>(), veff, eo, H->ent_atom.as<int32_t>(),
                                                 ent_beta_of<T>(H), C, nvec, X, ldx, Y, ldy, Z, ldz, coef);
    LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// optional per-kernel timing: HIP events recorded on the launch stream
// around every H X and KB-gather launch while enabled
// ---------------------------------------------------------------------------
struct KernelTimer {
    std::atomic<bool> on{false};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> spans[2];   // 0: H X, 1: KB gather
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        HIP_CHECK(hipEventCreate(&e));
        return e;
    }
    void recycle() {
        for (auto& v : spans) {
            for (auto& p : v) {
                pool.push_back(p.first);
                pool.push_back(p.second);
            }
            v.clear();
        }
    }
};
static KernelTimer g_timer;
static std::mutex g_timer_mu;   // guards the event pool and the spans

template <class F>
static void timed(int which, hipStream_t s, F&& launch) {
    if (!g_timer.on.load(std::memory_order_relaxed)) {
        launch();
        return;
    }
    hipEvent_t a, b;
    {
        std::lock_guard<std::mutex> lk(g_timer_mu);
        a = g_timer.get();
        b = g_timer.get();
    }
    HIP_CHECK(hipEventRecord(a, s));
    launch();
    HIP_CHECK(hipEventRecord(b, s));
    std::lock_guard<std::mutex> lk(g_timer_mu);
    g_timer.spans[which].emplace_back(a, b);
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <class T>
bool tiled_ok(const chf_ham* H, const void* X, int64_t ldx, const void* Y, int64_t ldy, const void* Z, int64_t ldz,
              int nvec) {
    constexpr int LN = Lane<T>::N;
    if (H->grid.ordering != CHF_ORDER_HILBERT) return false;
    if (nvec % LN || ldx % LN || ldy % LN || (Z && ldz % LN)) return false;
    if (int64_t(kBlockPts) * std::max(ldx, std::max(ldy, ldz)) * int64_t(sizeof(T)) >= (int64_t(1) << 30)) return false;
    const uintptr_t al = 8;
    if (uintptr_t(X) % al || uintptr_t(Y) % al || (Z && uintptr_t(Z) % al)) return false;
    return true;
}

// bytes of the KB coefficient scratch C [4 n_proj][nvec] of an H X launch
size_t kb_coef_bytes(const chf_ham* H, int nvec, size_t elem_bytes) {
    return size_t(std::max<int64_t>(1, H->proj.n_proj)) * 4 * size_t(nvec) * elem_bytes;
}

template <class T>
void hx_step(chf_ham* H, const T* X, int64_t ldx, T* Y, int64_t ldy, const T* Z, int64_t ldz, int nvec, double alpha,
             double shift, double beta, hipStream_t s, int force_kernel, bool lap_only, T* C_ext) {
    // the KB coefficients go to the handle's scratch (grown on demand), or to
    // the caller's C_ext (no allocation, no kernel timing)
    T* C = C_ext;
    if (!C) {
        H->kb_coef.ensure(kb_coef_bytes(H, nvec, sizeof(T)));
        C = H->kb_coef.as<T>();
    }
    auto run = [&](int which, auto&& launch) {
        if (C_ext) launch();
        else timed(which, s, launch);
    };
    if (H->proj.n_proj > 0 && !lap_only) run(1, [&] { launch_kb_gather<T>(H, X, ldx, nvec, C, s); });
    const bool tiled = force_kernel != 1 && tiled_ok<T>(H, X, ldx, Y, ldy, Z, ldz, nvec);
    if (tiled) {
        run(0, [&] { launch_hx_tiled<T>(H, X, ldx, Y, ldy, Z, ldz, nvec, C, alpha, shift, beta, s, lap_only); });
    } else {
        if (!H->has_nbr) fail(CHF_EUNSUPPORTED, "generic H X needs the neighbour table (keep_nbr) for this layout");
        run(0, [&] { launch_hx_generic<T>(H, X, ldx, Y, ldy, Z, ldz, nvec, C, alpha, shift, beta, s, lap_only); });
    }
}

// Degree-m scaled filter (CheFSI paragraph; the Zhou-Saad form).  With
// e = (b - a) / 2, c = (b + a) / 2 and sigma_k = T_{k-1}(t0) / T_k(t0),
// t0 = (a0 - c) / e, the normalised iterates Y_k = T_k((H - c) / e) X / T_k(t0)
// obey
//   Y_1 = (sigma_1 / e) (H - c) X,
//   Y_k = (2 sigma_k / e) (H - c) Y_{k-1} - sigma_{k-1} sigma_k Y_{k-2},
//   sigma_1 = e / (a0 - c), sigma_k = 1 / (2 / sigma_1 - sigma_{k-1}).
// Y_k overwrites Y_{k-2} in place (X for even k, the work block for odd k).
// The vectors are independent, so a work block narrower than the block is
// used column block by column block: min(nvec, ldw, max_cols) columns at a
// time (a multiple of 64, else of 4, when fewer than nvec, so that every
// block keeps the kernels' 16-byte alignment).  C_ext: KB-coefficient
// scratch of the caller for max_cols vectors (NULL: the handle's own).
template <class T>
void filter_run(chf_ham* H, T* X, int64_t ldx, T* W, int64_t ldw, int nvec, int m, double a, double b, double a0,
                hipStream_t s, int force_kernel, int64_t max_cols, T* C_ext) {
    const double e = (b - a) / 2, c = (b + a) / 2;
    const double sigma1 = e / (a0 - c);
    int64_t nb = std::min<int64_t>(nvec, std::min<int64_t>(ldw, max_cols));
    if (nb < nvec && nb >= 64) nb -= nb % 64;
    else if (nb < nvec && nb >= 4) nb -= nb % 4;
    for (int c0 = 0; c0 < nvec; c0 += int(nb)) {
        const int w = int(std::min<int64_t>(nb, nvec - c0));
        T* Xc = X + c0;
        double sigma = sigma1;
        hx_step<T>(H, Xc, ldx, W, ldw, nullptr, 0, w, sigma1 / e, c, 0.0, s, force_kernel, false, C_ext);
        for (int k = 2; k <= m; ++k) {
            const double sigma_next = 1.0 / (2.0 / sigma1 - sigma);
            const double alpha = 2.0 * sigma_next / e, beta = sigma * sigma_next;
            if (k % 2 == 0)
                hx_step<T>(H, W, ldw, Xc, ldx, Xc, ldx, w, alpha, c, beta, s, force_kernel, false, C_ext);
            else
                hx_step<T>(H, Xc, ldx, W, ldw, W, ldw, w, alpha, c, beta, s, force_kernel, false, C_ext);
            sigma = sigma_next;
        }
        if (m % 2 == 1)
            HIP_CHECK(hipMemcpy2DAsync(Xc, size_t(ldx) * sizeof(T), W, size_t(ldw) * sizeof(T), size_t(w) * sizeof(T),
                                       size_t(H->grid.n_rows), hipMemcpyDeviceToDevice, s));
    }
}

template void filter_run<float>(chf_ham*, float*, int64_t, float*, int64_t, int, int, double, double, double,
                                hipStream_t, int, int64_t, float*);
template void filter_run<double>(chf_ham*, double*, int64_t, double*, int64_t, int, int, double, double, double,
                                 hipStream_t, int, int64_t, double*);

// ---------------------------------------------------------------------------
// Allocation-free filter (chebyshev_filter_noalloc): the KB coefficients live
// in this fixed device array instead of the handle's scratch.  Each device
// the library runs on holds its own copy until the process ends; its address
// on a device is looked up once, with that device current, when the first
// Hamiltonian is built there (ham_build), and only that address is passed to
// kernels.  Calls that overlap on one device share the array and race.
// ---------------------------------------------------------------------------
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

void noalloc_scratch_init(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    CHF_REQUIRE(device >= 0 && device < kMaxDevices, "device index %d beyond %d", device, kMaxDevices);
    if (g_scratch_ptr[device]) return;
    void* p = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    CHF_REQUIRE(p != nullptr, "no device address for the filter scratch");
    g_scratch_ptr[device] = p;
}

template <class T>
void filter_run_noalloc(chf_ham* H, T* X, int64_t ldx, T* W, int64_t ldw, int nvec, int m, double a, double b,
                        double a0, hipStream_t s) {
    void* p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (H->device >= 0 && H->device < kMaxDevices) p = g_scratch_ptr[H->device];
    }
    if (!p) fail(CHF_EINVAL, "chebyshev_filter_noalloc: no scratch on device %d (no Hamiltonian built there)", H->device);
    // KB coefficients of one vector: 4 channels per projector atom
    const size_t per_vec = kb_coef_bytes(H, 1, sizeof(T));
    const int64_t max_cols = int64_t(kNoallocScratchBytes / per_vec);
    if (max_cols < 1)
        fail(CHF_EINVAL, "chebyshev_filter_noalloc: the KB coefficients of one vector (%zu bytes for %lld projector "
             "atoms) exceed the %zu-byte scratch", per_vec, (long long)H->proj.n_proj, kNoallocScratchBytes);
    filter_run<T>(H, X, ldx, W, ldw, nvec, m, a, b, a0, s, 0, max_cols, static_cast<T*>(p));
}

template void filter_run_noalloc<float>(chf_ham*, float*, int64_t, float*, int64_t, int, int, double, double, double,
                                        hipStream_t);
template void filter_run_noalloc<double>(chf_ham*, double*, int64_t, double*, int64_t, int, int, double, double,
                                         double, hipStream_t);

void timer_enable(int on) {
    std::lock_guard<std::mutex> lk(g_timer_mu);
    g_timer.recycle();
    g_timer.on.store(on != 0, std::memory_order_relaxed);
}

void timer_read(double* ms, int64_t* launches) {
    HIP_CHECK(hipDeviceSynchronize());
    std::lock_guard<std::mutex> lk(g_timer_mu);
    for (int w = 0; w < 2; ++w) {
        double t = 0;
        for (auto& p : g_timer.spans[w]) {
            float f = 0;
            HIP_CHECK(hipEventElapsedTime(&f, p.first, p.second));
            t += f;
        }
        ms[w] = t;
        launches[w] = int64_t(g_timer.spans[w].size());
    }
}

template void hx_step<float>(chf_ham*, const float*, int64_t, float*, int64_t, const float*, int64_t, int, double,
                             double, double, hipStream_t, int, bool, float*);
template void hx_step<double>(chf_ham*, const double*, int64_t, double*, int64_t, const double*, int64_t, int,
                              double, double, double, hipStream_t, int, bool, double*);
template void launch_kb_gather<float>(chf_ham*, const float*, int64_t, int, float*, hipStream_t);
template void launch_kb_gather<double>(chf_ham*, const double*, int64_t, int, double*, hipStream_t);

}  // namespace chf
