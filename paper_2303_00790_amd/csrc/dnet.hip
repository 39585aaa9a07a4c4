// Learned correction of the initial SCF density on gfx950: a 3-D U-Net
// (4 levels, 32 channels) trained and evaluated by hand-written kernels.
//
// The paper starts each SCF from a superposition of atomic densities; this
// network maps that superposition (on cubic patches of the real-space grid)
// to a correction towards the converged density, learned from densities the
// method itself produces.  Convolutions are implicit GEMMs on the BF16 MFMA
// (v_mfma_f32_16x16x16bf16_1k) with FP32 accumulation: BF16 weights and
// activations, FP32 master weights, pre-activations and gradients.
//
// Layout: activations channels-last [D][H][W][C]; weights [C_out][tap][C_in]
// with tap = (dz * 3 + dy) * 3 + dx (a single tap for the 1^3 output layer).
// Channel counts are padded to multiples of 4 (inputs) and 16 (outputs).
//
// Architecture (f = SiLU, up = nearest x2, [.,.] = channel concat):
//   e1 = f(c1b(f(c1a(x))))                      S^3
//   e2 = f(c2b(f(c2a(f(d1(e1))))))              (S/2)^3, d* stride 2
//   e3 = f(c3b(f(c3a(f(d2(e2))))))              (S/4)^3
//   b  = f(c4b(f(c4a(f(d3(e3))))))              (S/8)^3
//   g3 = f(c5b(f(c5a([f(u3(up(b))), e3]))))
//   g2 = f(c6b(f(c6a([f(u2(up(g3))), e2]))))
//   g1 = f(c7b(f(c7a([f(u1(up(g2))), e1]))))
//   y  = out(g1)                                 1^3 conv, no activation
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

namespace chf {
namespace dn {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16;

__device__ __host__ inline bf16 to_bf16(float f) {
    // round to nearest even
    const uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return bf16(u >> 16);   // inf / nan
    const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return bf16(r >> 16);
}
__device__ __host__ inline float from_bf16(bf16 b) {
    return __builtin_bit_cast(float, uint32_t(b) << 16);
}

__device__ inline float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ inline float silu_grad(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

struct Layer {
    int cin, cout;          // real channel counts
    int cin_p, cout_p;      // padded: multiple of 4 / 16
    int k, stride;          // kernel edge (3 or 1), stride (1 or 2)
    int64_t w_off, b_off;   // offsets into the master parameter vector (padded layout)
    bool act;
};

// ---------------------------------------------------------------------------
// forward: out[p][co] = b[co] + sum_{tap, ci} W[co][tap][ci] in[stride p + t - pad][ci]
// M = co (padded to 16 per block, 2 blocks max), N = output positions (16 per
// wave, 64 per workgroup), K = tap x ci in chunks of 16.  Input channels come
// from one or two tensors (channel concat).
// MFMA 16x16x16 bf16 operands: A(i, k) at lane i + 16 (k / 4), element k % 4;
// B(k, j) at lane j + 16 (k / 4), element k % 4; D(i, j): lane j + 16 (i / 4),
// register i % 4.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) conv_fwd_kernel(int Di, int Do, int cin0, int cin1, int cin_p, int cout, int cout_p,
                                                       int k, int stride, const bf16* __restrict__ in0,
                                                       const bf16* __restrict__ in1, const bf16* __restrict__ Wb,
                                                       const float* __restrict__ bias, float* __restrict__ zout,
                                                       bf16* __restrict__ yout, int act) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t npos = int64_t(Do) * Do * Do;
    const int64_t p0 = (int64_t(blockIdx.x) * 4 + wave) * 16;
    const int j = lane & 15, kq = lane >> 4;
    const int64_t p = p0 + j;
    const bool pok = p < npos;
    const int pz = pok ? int(p / (int64_t(Do) * Do)) : 0, py = pok ? int((p / Do) % Do) : 0, px = pok ? int(p % Do) : 0;
    const int pad = k / 2, ntap = k * k * k;
    const int K = ntap * cin_p;
    const int nrb = cout_p / 16;
    f4 acc[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    for (int kc = 0; kc < K; kc += 16) {
        const int kk = kc + 4 * kq;           // first of this lane's 4 k values
        s4 b = {0, 0, 0, 0};
        if (kk < K && pok) {
            const int tap = kk / cin_p, ci = kk % cin_p;
            const int dz = tap / (k * k), dy = (tap / k) % k, dx = tap % k;
            const int z = stride * pz + dz - pad, y = stride * py + dy - pad, x = stride * px + dx - pad;
            if (z >= 0 && z < Di && y >= 0 && y < Di && x >= 0 && x < Di) {
                const int64_t q = (int64_t(z) * Di + y) * Di + x;
                const bf16* src = ci < cin0 ? in0 + q * cin0 + ci : in1 + q * cin1 + (ci - cin0);
                if (ci < cin0 + cin1) b = *reinterpret_cast<const s4*>(src);
            }
        }
        for (int rb = 0; rb < nrb; ++rb) {
            s4 a = {0, 0, 0, 0};
            const int co = rb * 16 + j;
            if (kk < K) a = *reinterpret_cast<const s4*>(Wb + (int64_t(co) * ntap) * cin_p + kk);
            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[rb], 0, 0, 0);
        }
    }
    if (!pok) return;
    for (int rb = 0; rb < nrb; ++rb)
        for (int v = 0; v < 4; ++v) {
            const int co = rb * 16 + 4 * kq + v;
            if (co >= cout) continue;
            const float z = acc[rb][v] + bias[co];
            zout[p * cout + co] = z;
            yout[p * cout + co] = to_bf16(act ? silu(z) : z);
        }
}

// dZ = dY * f'(Z) (or dY when no activation), kept in FP32 and BF16
__global__ void act_back_kernel(int64_t n, const float* __restrict__ dy, const float* __restrict__ z, int act,
                                float* __restrict__ dz, bf16* __restrict__ dzb) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = act ? dy[i] * silu_grad(z[i]) : dy[i];
    dz[i] = g;
    dzb[i] = to_bf16(g);
}

// transposed copy of the weights for the data gradient: WT[ci][tap][co] (co padded to 4)
__global__ void weight_t_kernel(int cout, int cout_p4, int ntap, int cin_p, const float* __restrict__ W, bf16* __restrict__ WT) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t total = int64_t(cin_p) * ntap * cout_p4;
    if (idx >= total) return;
    const int co = int(idx % cout_p4);
    const int tap = int((idx / cout_p4) % ntap);
    const int ci = int(idx / (int64_t(cout_p4) * ntap));
    WT[idx] = co < cout ? to_bf16(W[(int64_t(co) * ntap + tap) * cin_p + ci]) : bf16(0);
}

// data gradient: dX[q][ci] = sum_{tap, co} dZ[p][co] W[co][tap][ci] with
// stride p + tap - pad = q.  M = ci, N = input positions, K = tap x co.
__global__ void __launch_bounds__(256) conv_bwd_data_kernel(int Di, int Do, int cin, int cin_rows, int cout, int cout_p4, int k,
                                                            int stride, const bf16* __restrict__ dzb,
                                                            const bf16* __restrict__ WT, float* __restrict__ dx) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t npos = int64_t(Di) * Di * Di;
    const int64_t q0 = (int64_t(blockIdx.x) * 4 + wave) * 16;
    const int j = lane & 15, kq = lane >> 4;
    const int64_t q = q0 + j;
    const bool qok = q < npos;
    const int qz = qok ? int(q / (int64_t(Di) * Di)) : 0, qy = qok ? int((q / Di) % Di) : 0, qx = qok ? int(q % Di) : 0;
    const int pad = k / 2, ntap = k * k * k;
    const int K = ntap * cout_p4;
    const int nrb = (cin_rows + 15) / 16;
    f4 acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    for (int kc = 0; kc < K; kc += 16) {
        const int kk = kc + 4 * kq;
        s4 b = {0, 0, 0, 0};
        int tap = 0;
        if (kk < K) tap = kk / cout_p4;
        const int co = kk % cout_p4;
        if (kk < K && qok) {
            const int dz = tap / (k * k), dy = (tap / k) % k, dx = tap % k;
            // output position p with stride p + d - pad = q
            const int nz = qz - dz + pad, ny = qy - dy + pad, nx = qx - dx + pad;
            if (nz >= 0 && ny >= 0 && nx >= 0 && nz % stride == 0 && ny % stride == 0 && nx % stride == 0) {
                const int z = nz / stride, y = ny / stride, x = nx / stride;
                if (z < Do && y < Do && x < Do) {
                    const int64_t p = (int64_t(z) * Do + y) * Do + x;
                    if (co + 3 < cout) {
                        b = *reinterpret_cast<const s4*>(dzb + p * cout + co);
                    } else {
                        for (int e = 0; e < 4; ++e) b[e] = co + e < cout ? short(dzb[p * cout + co + e]) : short(0);
                    }
                }
            }
        }
        for (int rb = 0; rb < nrb; ++rb) {
            s4 a = {0, 0, 0, 0};
            const int ci = rb * 16 + j;
            if (kk < K && ci < cin_rows) a = *reinterpret_cast<const s4*>(WT + (int64_t(ci) * ntap + tap) * cout_p4 + co);
            acc[rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[rb], 0, 0, 0);
        }
    }
    if (!qok) return;
    for (int rb = 0; rb < nrb; ++rb)
        for (int v = 0; v < 4; ++v) {
            const int ci = rb * 16 + 4 * kq + v;
            if (ci < cin) dx[q * cin + ci] = acc[rb][v];
        }
}

// weight gradient partials: dW[co][tap][ci] = sum_p dZ[p][co] X[stride p + t - pad][ci]
// M = co, N = (tap, ci) columns (16 per wave), K = output positions (this
// workgroup's slice, 16 per step).
__global__ void __launch_bounds__(256) conv_bwd_weight_kernel(int Di, int Do, int cin0, int cin1, int cin_p, int cout,
                                                              int k, int stride, const bf16* __restrict__ dzb,
                                                              const bf16* __restrict__ in0, const bf16* __restrict__ in1,
                                                              int64_t pos_per_split, float* __restrict__ part) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane & 15, kq = lane >> 4;
    const int ntap = k * k * k, pad = k / 2;
    const int ncol = ntap * cin_p;
    const int col = (blockIdx.x * 4 + wave) * 16 + j;
    const bool cok = col < ncol;
    const int tap = cok ? col / cin_p : 0, ci = cok ? col % cin_p : 0;
    const int dz = tap / (k * k), dy = (tap / k) % k, dx = tap % k;
    const int64_t npos = int64_t(Do) * Do * Do;
    const int64_t pb = int64_t(blockIdx.y) * pos_per_split, pe = min(npos, pb + pos_per_split);
    const int nrb = (cout + 15) / 16;
    f4 acc[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    for (int64_t pc = pb; pc < pe; pc += 16) {
        s4 b = {0, 0, 0, 0};
        s4 a[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
        for (int e = 0; e < 4; ++e) {
            const int64_t p = pc + 4 * kq + e;
            if (p >= pe) continue;
            const int pz = int(p / (int64_t(Do) * Do)), py = int((p / Do) % Do), px = int(p % Do);
            if (cok && ci < cin0 + cin1) {
                const int z = stride * pz + dz - pad, y = stride * py + dy - pad, x = stride * px + dx - pad;
                if (z >= 0 && z < Di && y >= 0 && y < Di && x >= 0 && x < Di) {
                    const int64_t q = (int64_t(z) * Di + y) * Di + x;
                    b[e] = short(ci < cin0 ? in0[q * cin0 + ci] : in1[q * cin1 + ci - cin0]);
                }
            }
            for (int rb = 0; rb < nrb; ++rb) {
                const int co = rb * 16 + j;
                if (co < cout) a[rb][e] = short(dzb[p * cout + co]);
            }
        }
        for (int rb = 0; rb < nrb; ++rb) acc[rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[rb], b, acc[rb], 0, 0, 0);
    }
    float* P = part + int64_t(blockIdx.y) * 32 * ncol;
    for (int rb = 0; rb < nrb; ++rb)
        for (int v = 0; v < 4; ++v) {
            const int co = rb * 16 + 4 * kq + v;
            if (co < cout && cok) P[int64_t(co) * ncol + col] = acc[rb][v];
        }
}

// grad[co][tap][ci] += sum over splits (fixed order); db[co] += sum_p dZ[p][co]
__global__ void wgrad_reduce_kernel(int cout, int ncol, int nsplit, const float* __restrict__ part, float* __restrict__ gw) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= int64_t(cout) * ncol) return;
    float s = 0.0f;
    for (int sp = 0; sp < nsplit; ++sp) s += part[int64_t(sp) * 32 * ncol + idx];
    gw[idx] += s;
}

__global__ void __launch_bounds__(256) bgrad_kernel(int64_t npos, int cout, const float* __restrict__ dz, float* __restrict__ gb) {
    const int co = blockIdx.x;
    __shared__ float sh[256];
    float s = 0.0f;
    for (int64_t p = threadIdx.x; p < npos; p += 256) s += dz[p * cout + co];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) gb[co] += sh[0];
}

__global__ void upsample_kernel(int Ds, int c, const bf16* __restrict__ src, bf16* __restrict__ dst) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int Dd = 2 * Ds;
    if (idx >= int64_t(Dd) * Dd * Dd * c) return;
    const int ch = int(idx % c);
    const int64_t q = idx / c;
    const int z = int(q / (int64_t(Dd) * Dd)), y = int((q / Dd) % Dd), x = int(q % Dd);
    dst[idx] = src[((int64_t(z / 2) * Ds + y / 2) * Ds + x / 2) * c + ch];
}

__global__ void upsample_back_kernel(int Ds, int c, const float* __restrict__ gd, float* __restrict__ gs) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= int64_t(Ds) * Ds * Ds * c) return;
    const int ch = int(idx % c);
    const int64_t q = idx / c;
    const int z = int(q / (int64_t(Ds) * Ds)), y = int((q / Ds) % Ds), x = int(q % Ds);
    const int Dd = 2 * Ds;
    float s = 0.0f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e) s += gd[((int64_t(2 * z + a) * Dd + 2 * y + b) * Dd + 2 * x + e) * c + ch];
    gs[idx] = s;
}

// out = a (+ b) with channel split: take channels [c0, c0 + cn) of a [n][ca]
__global__ void slice_add_kernel(int64_t n, int ca, int c0, int cn, const float* __restrict__ a, const float* __restrict__ b,
                                 float* __restrict__ out) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * cn) return;
    const int64_t p = idx / cn;
    const int ch = int(idx % cn);
    out[idx] = a[p * ca + c0 + ch] + (b ? b[idx] : 0.0f);
}

__global__ void input_kernel(int64_t n, const float* __restrict__ x, bf16* __restrict__ xb) {
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    xb[4 * p] = to_bf16(x[p]);
    xb[4 * p + 1] = 0;
    xb[4 * p + 2] = 0;
    xb[4 * p + 3] = 0;
}

__global__ void output_kernel(int64_t n, const float* __restrict__ z, float* __restrict__ y) {
    const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p < n) y[p] = z[p];
}

__global__ void cast_params_kernel(int64_t n, const float* __restrict__ w, bf16* __restrict__ wb) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = to_bf16(w[i]);
}

__global__ void adam_kernel(int64_t n, float* __restrict__ w, float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    g[i] = 0.0f;
}

// MSE loss partials and gradient dy = 2 (y - t) / n
__global__ void __launch_bounds__(256) mse_kernel(int64_t n, const float* __restrict__ y, const float* __restrict__ t,
                                                  float* __restrict__ dy, double* __restrict__ part) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const float d = y[i] - t[i];
        acc += double(d) * d;
        if (dy) dy[i] = 2.0f * d / float(n);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// patch of edge S from a box of edge D at offset (ox, oy, oz) under one of
// the 48 cubic symmetries: sym = perm * 8 + flips, perm indexes the 6 axis
// permutations, bit a of flips mirrors output axis a.  Out-of-box cells read 0.
__global__ void crop_kernel(int D, int S, int ox, int oy, int oz, int sym, const float* __restrict__ box,
                            float* __restrict__ patch) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= int64_t(S) * S * S) return;
    int c[3] = {int(idx % S), int((idx / S) % S), int(idx / (int64_t(S) * S))};   // x, y, z of the patch
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const int pm = (sym >> 3) % 6, fl = sym & 7;
    for (int a = 0; a < 3; ++a)
        if (fl & (1 << a)) c[a] = S - 1 - c[a];
    int s[3];
    for (int a = 0; a < 3; ++a) s[perms[pm][a]] = c[a];
    const int x = ox + s[0], y = oy + s[1], z = oz + s[2];
    float v = 0.0f;
    if (x >= 0 && y >= 0 && z >= 0 && x < D && y < D && z < D) v = box[(int64_t(z) * D + y) * D + x];
    patch[idx] = v;
}

__global__ void rows_to_box_kernel(int64_t n_rows, const int32_t* __restrict__ ijk4, const double* __restrict__ rows,
                                   const double* __restrict__ base, double scale, float* __restrict__ box, int D,
                                   int off) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n_rows || !ijk4[4 * r + 3]) return;
    const int x = ijk4[4 * r] + off, y = ijk4[4 * r + 1] + off, z = ijk4[4 * r + 2] + off;
    if (x < 0 || y < 0 || z < 0 || x >= D || y >= D || z >= D) return;
    const double v = base ? rows[r] - base[r] : rows[r];
    box[(int64_t(z) * D + y) * D + x] = float(scale * v);
}

__global__ void box_to_rows_kernel(int64_t n_rows, const int32_t* __restrict__ ijk4, const float* __restrict__ box, int D,
                                   int off, double inv_scale, const double* __restrict__ base, double* __restrict__ out) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    if (!ijk4[4 * r + 3]) {
        out[r] = 0.0;
        return;
    }
    const int x = ijk4[4 * r] + off, y = ijk4[4 * r + 1] + off, z = ijk4[4 * r + 2] + off;
    double v = base ? base[r] : 0.0;
    if (x >= 0 && y >= 0 && z >= 0 && x < D && y < D && z < D) v += inv_scale * double(box[(int64_t(z) * D + y) * D + x]);
    out[r] = v;
}

// one pass of a separable, truncated, normalised Gaussian along one axis of
// a cubic box (x fastest), zero outside: out[i] = sum_k g[k + r] in[i + k e]
__global__ void blur_pass_kernel(int D, int axis, int r, const float* __restrict__ g, const float* __restrict__ in,
                                 float* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = int64_t(D) * D * D;
    if (i >= n) return;
    const int x = int(i % D), y = int((i / D) % D), z = int(i / (int64_t(D) * D));
    const int c = axis == 0 ? x : (axis == 1 ? y : z);
    const int64_t stride = axis == 0 ? 1 : (axis == 1 ? D : int64_t(D) * D);
    float acc = 0.f;
    for (int k = -r; k <= r; ++k) {
        const int q = c + k;
        if (q >= 0 && q < D) acc = fmaf(g[k + r], in[i + k * stride], acc);
    }
    out[i] = acc;
}

__global__ void sub_kernel(int64_t n, const float* __restrict__ a, const float* __restrict__ b, float* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] - b[i];
}

static uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

}  // namespace dn
}  // namespace chf

using namespace chf;
using namespace chf::dn;

struct dnet {
    int C = 32;
    std::vector<Layer> L;
    int64_t n_params = 0;
    DevBuf w, g, m, v;            // FP32 master params, grads, Adam moments
    DevBuf wb;                    // BF16 copy of the weights
    DevBuf wt;                    // BF16 transposed weights (scratch, one layer)
    DevBuf part;                  // weight-gradient partials / loss partials
    int S = 0;                    // patch edge the activation buffers are sized for
    // activation tape: for each layer the input pointer(s) and Z / Y buffers
    struct Act {
        DevBuf z, y;
        int D = 0;                // output edge
    };
    std::vector<std::unique_ptr<Act>> act;
    DevBuf xin;                   // BF16 input [S^3][4]
    DevBuf up[3];                 // upsampled inputs of u3, u2, u1
    DevBuf gA, gB, gC, gD;        // FP32 gradient scratch
    DevBuf dzb;                   // BF16 dZ
    hipStream_t stream = nullptr;
};

namespace {

enum {
    C1A, C1B, D1, C2A, C2B, D2, C3A, C3B, D3, C4A, C4B, U3, C5A, C5B, U2, C6A, C6B, U1, C7A, C7B, OUT, NLAYER
};

void make_layers(dnet* N) {
    const int C = N->C;
    struct Spec {
        int cin, cout, k, stride;
        bool act;
    };
    const Spec sp[NLAYER] = {{1, C, 3, 1, true},     {C, C, 3, 1, true},     {C, C, 3, 2, true}, {C, C, 3, 1, true},
                             {C, C, 3, 1, true},     {C, C, 3, 2, true},     {C, C, 3, 1, true}, {C, C, 3, 1, true},
                             {C, C, 3, 2, true},     {C, C, 3, 1, true},     {C, C, 3, 1, true}, {C, C, 3, 1, true},
                             {2 * C, C, 3, 1, true}, {C, C, 3, 1, true},     {C, C, 3, 1, true}, {2 * C, C, 3, 1, true},
                             {C, C, 3, 1, true},     {C, C, 3, 1, true},     {2 * C, C, 3, 1, true},
                             {C, C, 3, 1, true},     {C, 1, 1, 1, false}};
    int64_t off = 0;
    for (int i = 0; i < NLAYER; ++i) {
        Layer l;
        l.cin = sp[i].cin;
        l.cout = sp[i].cout;
        l.cin_p = ((l.cin + 3) / 4) * 4;
        l.cout_p = ((l.cout + 15) / 16) * 16;
        l.k = sp[i].k;
        l.stride = sp[i].stride;
        l.act = sp[i].act;
        l.w_off = off;
        off += int64_t(l.cout_p) * l.k * l.k * l.k * l.cin_p;
        l.b_off = off;
        off += l.cout_p;
        N->L.push_back(l);
    }
    N->n_params = off;
}

unsigned nb(int64_t n) { return unsigned((n + 255) / 256); }

// edge of the output of layer i for patch edge S: encoder levels S, S/2, S/4,
// S/8 (the stride-2 layer opens its level), decoder levels S/4, S/2, S (the
// upsampling conv opens its level), and the 1^3 output layer at S
int out_edge(int i, int S) {
    static const int div[NLAYER] = {1, 1,          // c1a c1b
                                    2, 2, 2,       // d1 c2a c2b
                                    4, 4, 4,       // d2 c3a c3b
                                    8, 8, 8,       // d3 c4a c4b
                                    4, 4, 4,       // u3 c5a c5b
                                    2, 2, 2,       // u2 c6a c6b
                                    1, 1, 1,       // u1 c7a c7b
                                    1};            // out
    return S / div[i];
}

void ensure_buffers(dnet* N, int S) {
    if (N->S == S) return;
    const int C = N->C;
    N->act.clear();
    for (int i = 0; i < NLAYER; ++i) {
        const int D = out_edge(i, S);
        const int64_t n = int64_t(D) * D * D * N->L[i].cout;
        N->act.emplace_back(new dnet::Act);
        N->act[i]->D = D;
        N->act[i]->z.alloc(size_t(n) * sizeof(float));
        N->act[i]->y.alloc(size_t(n) * sizeof(bf16));
    }
    N->xin.alloc(size_t(S) * S * S * 4 * sizeof(bf16));
    N->up[0].alloc(size_t(S / 4) * (S / 4) * (S / 4) * C * sizeof(bf16));
    N->up[1].alloc(size_t(S / 2) * (S / 2) * (S / 2) * C * sizeof(bf16));
    N->up[2].alloc(size_t(S) * S * S * C * sizeof(bf16));
    const size_t big = size_t(S) * S * S * 2 * C * sizeof(float);
    N->gA.alloc(big);
    N->gB.alloc(big);
    N->gC.alloc(big);
    N->gD.alloc(big);
    N->dzb.alloc(size_t(S) * S * S * C * sizeof(bf16));
    N->S = S;
}

void conv_forward(dnet* N, int i, int Di, const bf16* in0, int c0, const bf16* in1, int c1, hipStream_t s) {
    const Layer& l = N->L[i];
    const int Do = N->act[i]->D;
    const int64_t npos = int64_t(Do) * Do * Do;
    conv_fwd_kernel<<<unsigned((npos + 63) / 64), 256, 0, s>>>(
        Di, Do, c0, c1, l.cin_p, l.cout, l.cout_p, l.k, l.stride, in0, in1, N->wb.as<bf16>() + l.w_off,
        N->w.as<float>() + l.b_off, N->act[i]->z.as<float>(), N->act[i]->y.as<bf16>(), l.act ? 1 : 0);
    LAUNCH_CHECK();
}

// backward through layer i: dy (FP32, [Do^3][cout]) -> parameter grads and
// (optionally) dx (FP32, [Di^3][cin])
void conv_backward(dnet* N, int i, int Di, const bf16* in0, int c0, const bf16* in1, int c1, const float* dy, float* dx,
                   hipStream_t s) {
    const Layer& l = N->L[i];
    const int Do = N->act[i]->D;
    const int64_t npos = int64_t(Do) * Do * Do;
    const int ntap = l.k * l.k * l.k;
    float* dz = N->gD.as<float>();
    act_back_kernel<<<nb(npos * l.cout), 256, 0, s>>>(npos * l.cout, dy, N->act[i]->z.as<float>(), l.act ? 1 : 0, dz,
                                                      N->dzb.as<bf16>());
    LAUNCH_CHECK();
    // weight gradient: split-K over output positions
    const int ncol = ntap * l.cin_p;
    const int ncb = (ncol + 63) / 64;
    int nsplit = int(std::min<int64_t>(256, std::max<int64_t>(1, npos / 1024)));
    const int64_t per = ((npos + nsplit - 1) / nsplit + 15) / 16 * 16;
    nsplit = int((npos + per - 1) / per);
    N->part.ensure(size_t(nsplit) * 32 * ncol * sizeof(float));
    conv_bwd_weight_kernel<<<dim3(ncb, nsplit), 256, 0, s>>>(Di, Do, c0, c1, l.cin_p, l.cout, l.k, l.stride,
                                                             N->dzb.as<bf16>(), in0, in1, per, N->part.as<float>());
    LAUNCH_CHECK();
    wgrad_reduce_kernel<<<nb(int64_t(l.cout) * ncol), 256, 0, s>>>(l.cout, ncol, nsplit, N->part.as<float>(),
                                                                  N->g.as<float>() + l.w_off);
    LAUNCH_CHECK();
    bgrad_kernel<<<l.cout, 256, 0, s>>>(npos, l.cout, dz, N->g.as<float>() + l.b_off);
    LAUNCH_CHECK();
    if (!dx) return;
    const int cout_p4 = ((l.cout + 3) / 4) * 4;
    const int64_t nwt = int64_t(l.cin_p) * ntap * cout_p4;
    N->wt.ensure(size_t(nwt) * sizeof(bf16));
    weight_t_kernel<<<nb(nwt), 256, 0, s>>>(l.cout, cout_p4, ntap, l.cin_p, N->w.as<float>() + l.w_off, N->wt.as<bf16>());
    LAUNCH_CHECK();
    const int64_t nin = int64_t(Di) * Di * Di;
    conv_bwd_data_kernel<<<unsigned((nin + 63) / 64), 256, 0, s>>>(Di, Do, l.cin, l.cin_p, l.cout, cout_p4, l.k, l.stride,
                                                                   N->dzb.as<bf16>(), N->wt.as<bf16>(), dx);
    LAUNCH_CHECK();
}

template <class F>
int dguard(F&& f) {
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

}  // namespace

extern "C" {

int dnet_create(int channels, uint64_t seed, dnet** out) {
    return dguard([&] {
        if (!out) fail(CHF_EINVAL, "dnet_create: null out");
        *out = nullptr;
        if (channels < 4 || channels > 32 || channels % 4) fail(CHF_EINVAL, "dnet_create: channels must be 4..32, multiple of 4");
        auto N = std::make_unique<dnet>();
        N->C = channels;
        make_layers(N.get());
        // He-normal weights (Box-Muller over splitmix64), zero biases, zero
        // output layer so the untrained network predicts no correction
        std::vector<float> h(size_t(N->n_params), 0.0f);
        uint64_t st = seed;
        for (int i = 0; i < NLAYER; ++i) {
            const Layer& l = N->L[i];
            if (i == OUT) continue;
            const int ntap = l.k * l.k * l.k;
            const double sd = std::sqrt(2.0 / (double(l.cin) * ntap));
            for (int co = 0; co < l.cout; ++co)
                for (int t = 0; t < ntap; ++t)
                    for (int ci = 0; ci < l.cin; ++ci) {
                        const double u1 = (double(splitmix(st) >> 11) + 0.5) / 9007199254740992.0;
                        const double u2 = double(splitmix(st) >> 11) / 9007199254740992.0;
                        const double z = std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * 3.14159265358979323846 * u2);
                        h[size_t(l.w_off + (int64_t(co) * ntap + t) * l.cin_p + ci)] = float(sd * z);
                    }
        }
        N->w.alloc(size_t(N->n_params) * sizeof(float));
        N->g.alloc(size_t(N->n_params) * sizeof(float));
        N->m.alloc(size_t(N->n_params) * sizeof(float));
        N->v.alloc(size_t(N->n_params) * sizeof(float));
        N->wb.alloc(size_t(N->n_params) * sizeof(bf16));
        HIP_CHECK(hipMemcpy(N->w.p, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
        HIP_CHECK(hipMemset(N->g.p, 0, size_t(N->n_params) * sizeof(float)));
        HIP_CHECK(hipMemset(N->m.p, 0, size_t(N->n_params) * sizeof(float)));
        HIP_CHECK(hipMemset(N->v.p, 0, size_t(N->n_params) * sizeof(float)));
        *out = N.release();
    });
}

int dnet_destroy(dnet* N) {
    if (N) {
        (void)hipDeviceSynchronize();
        delete N;
    }
    return CHF_OK;
}

int dnet_param_count(const dnet* N, int64_t* n) {
    return dguard([&] {
        if (!N || !n) fail(CHF_EINVAL, "dnet_param_count: null argument");
        *n = N->n_params;
    });
}

int dnet_layer_info(const dnet* N, int layer, int* info6, int64_t* offsets2) {
    return dguard([&] {
        if (!N || !info6 || !offsets2 || layer < 0 || layer >= NLAYER) fail(CHF_EINVAL, "dnet_layer_info: bad argument");
        const Layer& l = N->L[size_t(layer)];
        info6[0] = l.cin;
        info6[1] = l.cout;
        info6[2] = l.cin_p;
        info6[3] = l.cout_p;
        info6[4] = l.k;
        info6[5] = l.stride;
        offsets2[0] = l.w_off;
        offsets2[1] = l.b_off;
    });
}

int dnet_plan(int S, int* edges) {
    return dguard([&] {
        if (!edges || S < 8 || S % 8) fail(CHF_EINVAL, "dnet_plan: S must be a positive multiple of 8");
        for (int i = 0; i < NLAYER; ++i) edges[i] = out_edge(i, S);
    });
}

int dnet_get_params(const dnet* N, float* host) {
    return dguard([&] {
        if (!N || !host) fail(CHF_EINVAL, "dnet_get_params: null argument");
        HIP_CHECK(hipDeviceSynchronize());
        HIP_CHECK(hipMemcpy(host, N->w.p, size_t(N->n_params) * sizeof(float), hipMemcpyDeviceToHost));
    });
}

int dnet_set_params(dnet* N, const float* host) {
    return dguard([&] {
        if (!N || !host) fail(CHF_EINVAL, "dnet_set_params: null argument");
        HIP_CHECK(hipDeviceSynchronize());
        HIP_CHECK(hipMemcpy(N->w.p, host, size_t(N->n_params) * sizeof(float), hipMemcpyHostToDevice));
    });
}

int dnet_forward(dnet* N, const float* x, int S, float* y, void* stream) {
    return dguard([&] {
        if (!N || !x || !y) fail(CHF_EINVAL, "dnet_forward: null argument");
        if (S < 8 || S % 8 || S > 512) fail(CHF_EINVAL, "dnet_forward: patch edge must be a multiple of 8 in [8, 512]");
        hipStream_t s = static_cast<hipStream_t>(stream);
        N->stream = s;
        ensure_buffers(N, S);
        const int C = N->C;
        cast_params_kernel<<<nb(N->n_params), 256, 0, s>>>(N->n_params, N->w.as<float>(), N->wb.as<bf16>());
        LAUNCH_CHECK();
        const int64_t n = int64_t(S) * S * S;
        input_kernel<<<nb(n), 256, 0, s>>>(n, x, N->xin.as<bf16>());
        LAUNCH_CHECK();
        auto Y = [&](int i) { return N->act[i]->y.as<bf16>(); };
        conv_forward(N, C1A, S, N->xin.as<bf16>(), 4, nullptr, 0, s);
        conv_forward(N, C1B, S, Y(C1A), C, nullptr, 0, s);
        conv_forward(N, D1, S, Y(C1B), C, nullptr, 0, s);
        conv_forward(N, C2A, S / 2, Y(D1), C, nullptr, 0, s);
        conv_forward(N, C2B, S / 2, Y(C2A), C, nullptr, 0, s);
        conv_forward(N, D2, S / 2, Y(C2B), C, nullptr, 0, s);
        conv_forward(N, C3A, S / 4, Y(D2), C, nullptr, 0, s);
        conv_forward(N, C3B, S / 4, Y(C3A), C, nullptr, 0, s);
        conv_forward(N, D3, S / 4, Y(C3B), C, nullptr, 0, s);
        conv_forward(N, C4A, S / 8, Y(D3), C, nullptr, 0, s);
        conv_forward(N, C4B, S / 8, Y(C4A), C, nullptr, 0, s);
        const int enc[3] = {C3B, C2B, C1B}, upl[3] = {U3, U2, U1}, ca[3] = {C5A, C6A, C7A}, cb[3] = {C5B, C6B, C7B};
        int prev = C4B;
        for (int lvl = 0; lvl < 3; ++lvl) {
            const int Ds = N->act[prev]->D, Dd = 2 * Ds;
            upsample_kernel<<<nb(int64_t(Dd) * Dd * Dd * C), 256, 0, s>>>(Ds, C, Y(prev), N->up[lvl].as<bf16>());
            LAUNCH_CHECK();
            conv_forward(N, upl[lvl], Dd, N->up[lvl].as<bf16>(), C, nullptr, 0, s);
            conv_forward(N, ca[lvl], Dd, Y(upl[lvl]), C, Y(enc[lvl]), C, s);
            conv_forward(N, cb[lvl], Dd, Y(ca[lvl]), C, nullptr, 0, s);
            prev = cb[lvl];
        }
        conv_forward(N, OUT, S, Y(C7B), C, nullptr, 0, s);
        output_kernel<<<nb(n), 256, 0, s>>>(n, N->act[OUT]->z.as<float>(), y);
        LAUNCH_CHECK();
    });
}

int dnet_backward(dnet* N, const float* dy, void* stream) {
    return dguard([&] {
        if (!N || !dy) fail(CHF_EINVAL, "dnet_backward: null argument");
        if (N->S == 0) fail(CHF_EINVAL, "dnet_backward: call dnet_forward first");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int S = N->S, C = N->C;
        auto Y = [&](int i) { return N->act[i]->y.as<bf16>(); };
        float* a = N->gA.as<float>();
        float* b = N->gB.as<float>();
        float* c = N->gC.as<float>();
        // out layer: input g1 = Y(C7B)
        conv_backward(N, OUT, S, Y(C7B), C, nullptr, 0, dy, a, s);   // a = dL/d g1
        // decoder levels (innermost last): keep the skip gradients
        float* skip[3] = {nullptr, nullptr, nullptr};
        const int enc[3] = {C3B, C2B, C1B}, upl[3] = {U3, U2, U1}, ca[3] = {C5A, C6A, C7A}, cb[3] = {C5B, C6B, C7B};
        const int prevl[3] = {C4B, C5B, C6B};
        std::vector<std::unique_ptr<DevBuf>> keep;
        for (int lvl = 2; lvl >= 0; --lvl) {
            const int Dd = N->act[cb[lvl]]->D, Ds = Dd / 2;
            const int64_t nd = int64_t(Dd) * Dd * Dd;
            conv_backward(N, cb[lvl], Dd, Y(ca[lvl]), C, nullptr, 0, a, b, s);             // b = dL/d Y(ca)
            conv_backward(N, ca[lvl], Dd, Y(upl[lvl]), C, Y(enc[lvl]), C, b, c, s);         // c = dL/d concat [nd][2C]
            keep.emplace_back(new DevBuf);
            keep.back()->alloc(size_t(nd) * C * sizeof(float));
            skip[lvl] = keep.back()->as<float>();
            slice_add_kernel<<<nb(nd * C), 256, 0, s>>>(nd, 2 * C, C, C, c, nullptr, skip[lvl]);  // encoder part
            LAUNCH_CHECK();
            slice_add_kernel<<<nb(nd * C), 256, 0, s>>>(nd, 2 * C, 0, C, c, nullptr, b);          // upsampled part
            LAUNCH_CHECK();
            conv_backward(N, upl[lvl], Dd, N->up[lvl].as<bf16>(), C, nullptr, 0, b, c, s);  // c = dL/d up(prev)
            upsample_back_kernel<<<nb(int64_t(Ds) * Ds * Ds * C), 256, 0, s>>>(Ds, C, c, a);  // a = dL/d Y(prev)
            LAUNCH_CHECK();
            (void)prevl;
        }
        // encoder: a = dL/d Y(C4B)
        conv_backward(N, C4B, S / 8, Y(C4A), C, nullptr, 0, a, b, s);
        conv_backward(N, C4A, S / 8, Y(D3), C, nullptr, 0, b, a, s);
        conv_backward(N, D3, S / 4, Y(C3B), C, nullptr, 0, a, b, s);                      // b = dL/d e3 (down path)
        int64_t n3 = int64_t(S / 4) * (S / 4) * (S / 4);
        slice_add_kernel<<<nb(n3 * C), 256, 0, s>>>(n3, C, 0, C, b, skip[0], a);
        LAUNCH_CHECK();
        conv_backward(N, C3B, S / 4, Y(C3A), C, nullptr, 0, a, b, s);
        conv_backward(N, C3A, S / 4, Y(D2), C, nullptr, 0, b, a, s);
        conv_backward(N, D2, S / 2, Y(C2B), C, nullptr, 0, a, b, s);
        int64_t n2 = int64_t(S / 2) * (S / 2) * (S / 2);
        slice_add_kernel<<<nb(n2 * C), 256, 0, s>>>(n2, C, 0, C, b, skip[1], a);
        LAUNCH_CHECK();
        conv_backward(N, C2B, S / 2, Y(C2A), C, nullptr, 0, a, b, s);
        conv_backward(N, C2A, S / 2, Y(D1), C, nullptr, 0, b, a, s);
        conv_backward(N, D1, S, Y(C1B), C, nullptr, 0, a, b, s);
        int64_t n1 = int64_t(S) * S * S;
        slice_add_kernel<<<nb(n1 * C), 256, 0, s>>>(n1, C, 0, C, b, skip[2], a);
        LAUNCH_CHECK();
        conv_backward(N, C1B, S, Y(C1A), C, nullptr, 0, a, b, s);
        conv_backward(N, C1A, S, N->xin.as<bf16>(), 4, nullptr, 0, b, nullptr, s);
        HIP_CHECK(hipStreamSynchronize(s));   // scratch buffers in `keep` are released below
    });
}

int dnet_get_grads(const dnet* N, float* host) {
    return dguard([&] {
        if (!N || !host) fail(CHF_EINVAL, "dnet_get_grads: null argument");
        HIP_CHECK(hipDeviceSynchronize());
        HIP_CHECK(hipMemcpy(host, N->g.p, size_t(N->n_params) * sizeof(float), hipMemcpyDeviceToHost));
    });
}

int dnet_adam(dnet* N, float lr, int step, void* stream) {
    return dguard([&] {
        if (!N || step < 1 || !(lr > 0)) fail(CHF_EINVAL, "dnet_adam: bad argument");
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.0f - std::pow(b1, float(step)), c2 = 1.0f - std::pow(b2, float(step));
        adam_kernel<<<nb(N->n_params), 256, 0, static_cast<hipStream_t>(stream)>>>(
            N->n_params, N->w.as<float>(), N->g.as<float>(), N->m.as<float>(), N->v.as<float>(), lr, b1, b2, 1e-8f, c1, c2);
        LAUNCH_CHECK();
    });
}

int dnet_mse(dnet* N, const float* y, const float* t, int64_t n, double* loss_host, float* dy, void* stream) {
    return dguard([&] {
        if (!N || !y || !t || !loss_host || n < 1) fail(CHF_EINVAL, "dnet_mse: bad argument");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int blocks = int(std::min<int64_t>(1024, (n + 255) / 256));
        N->part.ensure(size_t(blocks + 1) * sizeof(double));
        double* part = reinterpret_cast<double*>(N->part.p);
        mse_kernel<<<blocks, 256, 0, s>>>(n, y, t, dy, part);
        LAUNCH_CHECK();
        std::vector<double> h(static_cast<size_t>(blocks));
        HIP_CHECK(hipMemcpyAsync(h.data(), part, size_t(blocks) * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        double tot = 0;
        for (double v : h) tot += v;
        *loss_host = tot / double(n);
    });
}

int chf_rows_to_box(chf_ham* H, const double* rows, const double* base, double scale, float* box, int D, int off,
                    void* stream) {
    return dguard([&] {
        if (!H || !rows || !box || D < 1) fail(CHF_EINVAL, "chf_rows_to_box: bad argument");
        hipStream_t s = static_cast<hipStream_t>(stream);
        HIP_CHECK(hipMemsetAsync(box, 0, size_t(D) * D * D * sizeof(float), s));
        rows_to_box_kernel<<<nb(H->grid.n_rows), 256, 0, s>>>(H->grid.n_rows, H->row_ijk4.as<int32_t>(), rows, base,
                                                              scale, box, D, off);
        LAUNCH_CHECK();
    });
}

int chf_box_to_rows(chf_ham* H, const float* box, int D, int off, double scale, const double* base, double* out,
                    void* stream) {
    return dguard([&] {
        if (!H || !box || !out || D < 1 || !(scale != 0)) fail(CHF_EINVAL, "chf_box_to_rows: bad argument");
        box_to_rows_kernel<<<nb(H->grid.n_rows), 256, 0, static_cast<hipStream_t>(stream)>>>(
            H->grid.n_rows, H->row_ijk4.as<int32_t>(), box, D, off, 1.0 / scale, base, out);
        LAUNCH_CHECK();
    });
}

int dnet_highpass(const float* box, int D, double sigma, float* out, float* work, void* stream) {
    return dguard([&] {
        if (!box || !out || !work || D < 1 || !(sigma > 0) || sigma > 64) fail(CHF_EINVAL, "dnet_highpass: bad argument");
        const int r = int(std::ceil(3.0 * sigma));
        std::vector<float> g(size_t(2 * r + 1));
        double tot = 0;
        for (int k = -r; k <= r; ++k) tot += std::exp(-double(k) * k / (2.0 * sigma * sigma));
        for (int k = -r; k <= r; ++k) g[size_t(k + r)] = float(std::exp(-double(k) * k / (2.0 * sigma * sigma)) / tot);
        hipStream_t s = static_cast<hipStream_t>(stream);
        DevBuf gd;
        upload(gd, g, s);
        const int64_t n = int64_t(D) * D * D;
        float* t1 = work;
        float* t2 = work + n;
        blur_pass_kernel<<<nb(n), 256, 0, s>>>(D, 0, r, gd.as<float>(), box, t1);
        blur_pass_kernel<<<nb(n), 256, 0, s>>>(D, 1, r, gd.as<float>(), t1, t2);
        blur_pass_kernel<<<nb(n), 256, 0, s>>>(D, 2, r, gd.as<float>(), t2, t1);
        sub_kernel<<<nb(n), 256, 0, s>>>(n, box, t1, out);
        LAUNCH_CHECK();
        HIP_CHECK(hipStreamSynchronize(s));   // the weights buffer is freed on return
    });
}

int dnet_crop(const float* box, int D, int S, int ox, int oy, int oz, int sym, float* patch, void* stream) {
    return dguard([&] {
        if (!box || !patch || D < 1 || S < 1 || sym < 0 || sym >= 48) fail(CHF_EINVAL, "dnet_crop: bad argument");
        crop_kernel<<<nb(int64_t(S) * S * S), 256, 0, static_cast<hipStream_t>(stream)>>>(D, S, ox, oy, oz, sym, box, patch);
        LAUNCH_CHECK();
    });
}

}  // extern "C"
