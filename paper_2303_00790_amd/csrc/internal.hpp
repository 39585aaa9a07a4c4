// Internal declarations of the ChFSI library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <atomic>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/chfsi.h"

namespace chf {

// ---------------------------------------------------------------------------
// errors: every C entry point converts these into a status code + message
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(int code, const char* fmt, ...);
void set_last_error(const char* msg);

#define CHF_REQUIRE(cond, ...)                                         \
    do {                                                               \
        if (!(cond)) ::chf::fail(CHF_EINVAL, __VA_ARGS__);             \
    } while (0)

#define HIP_CHECK(expr)                                                             \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess)                                                       \
            ::chf::fail(CHF_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                        \
    } while (0)

#define LAUNCH_CHECK() HIP_CHECK(hipGetLastError())

#define ROCBLAS_CHECK(expr)                                                         \
    do {                                                                            \
        rocblas_status s_ = (expr);                                                 \
        if (s_ != rocblas_status_success)                                           \
            ::chf::fail(CHF_EHIP, "%s failed: %s", #expr, rocblas_status_to_string(s_)); \
    } while (0)

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
// device allocations made by the library so far (all handles, all devices)
inline std::atomic<int64_t> g_device_allocations{0};

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t n) {
        release();
        if (n == 0) return;
        if (hipMalloc(&p, n) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            fail(CHF_ENOMEM, "device allocation of %zu bytes failed", n);
        }
        bytes = n;
        g_device_allocations.fetch_add(1, std::memory_order_relaxed);
    }
    void ensure(size_t n) {
        if (n > bytes) alloc(n);
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

template <class T>
void upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
    b.alloc(v.size() * sizeof(T));
    if (!v.empty()) HIP_CHECK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// ---------------------------------------------------------------------------
// host-side grid / ordering / tables (host_grid.cpp)
// ---------------------------------------------------------------------------
constexpr int kBlock = 8;
constexpr int kBlockPts = 512;
constexpr int kHalf = 6;          // stencil half width (12th order)
constexpr int kNbr = 36;          // neighbours per point

struct HostGrid {
    double h = 0, radius = 0;
    int ordering = 0;
    int n_r = 0;            // floor(radius / h)
    int nb = 0;             // blocks per edge (Hilbert)
    int64_t n = 0;          // inside points
    int64_t n_rows = 0;
    int64_t n_blocks = 0;
    std::vector<int32_t> ijk;           // [n][3] by rank
    std::vector<int64_t> row_of_rank;   // [n]
    std::vector<int32_t> rank_of_row;   // [n_rows], -1 = padding
    std::vector<int32_t> blocks;        // [n_blocks][3] block coordinates by slot
    std::vector<int32_t> block_nbr;     // [n_blocks][6] face neighbours (-x,+x,-y,+y,-z,+z), -1 none
    std::vector<uint64_t> block_mask;   // [n_blocks][8] inside bits per local index
    std::vector<int32_t> slot_of_block; // [nb^3] (Hilbert), -1 empty

    // row of integer point (i, j, k) or -1 when outside
    int64_t row_of(int i, int j, int k) const;
    bool inside(int i, int j, int k) const;
    int64_t thr = 0;
    std::vector<int32_t> lex_cube;      // lexicographic: rank by cube index (only when needed)
};

void build_grid(HostGrid& g, double h, double radius, int ordering);
uint64_t hilbert_index3(uint32_t x, uint32_t y, uint32_t z, int nbits);
// per-row neighbour rows [n_rows][36] (-1 outside / padding rows all -1)
void build_row_neighbours(const HostGrid& g, std::vector<int32_t>& nbr_rows);

struct HostProj {
    int64_t n_proj = 0;                 // projector atoms (Si)
    std::vector<int32_t> atom_index;    // [n_proj] index into the atom list
    // per atom support (gather): rows ascending
    std::vector<int64_t> sup_off;       // [n_proj + 1]
    std::vector<int32_t> sup_row;       // [pairs]
    std::vector<double> sup_beta;       // [pairs][4] (s, px, py, pz), unscaled
    // per row entries (scatter): atoms ascending
    std::vector<int64_t> ent_off;       // [n_rows + 1]
    std::vector<int32_t> ent_atom;      // [pairs] projector-atom index
    std::vector<double> ent_beta;       // [pairs][4]
    // blockwise view (Hilbert layout): atoms touching each 8^3 block and the
    // slot of every row entry's atom in its block's list
    std::vector<int64_t> blk_atom_off;  // [n_blocks + 1]
    std::vector<int32_t> blk_atoms;     // projector-atom indices, ascending per block
    std::vector<uint8_t> ent_slot;      // [pairs]
    int max_block_atoms = 0;
};

void build_block_atoms(const HostGrid& g, HostProj& P);

void build_projectors(const HostGrid& g, const chf_atoms& atoms, const chf_pp& pp, HostProj& out);

// ---------------------------------------------------------------------------
// device-side objects
// ---------------------------------------------------------------------------
}  // namespace chf

struct chf_ham {
    int device = 0;
    chf::HostGrid grid;
    chf::HostProj proj;
    double h = 0;
    double coef[7] = {};        // -1/2 c_k / h^2
    // device tables
    chf::DevBuf nbr_rows;       // int32 [n_rows][36] (optional)
    chf::DevBuf block_nbr;      // int32 [n_blocks][6]
    chf::DevBuf block_mask;     // uint64 [n_blocks][8]
    chf::DevBuf row_inside;     // uint8 [n_rows]
    chf::DevBuf row_ijk4;       // int32 [n_rows][4]: i, j, k, inside flag
    chf::DevBuf vloc;           // double [n_rows]
    chf::DevBuf veff64;         // double [n_rows]
    chf::DevBuf veff32;         // float  [n_rows]
    chf::DevBuf sup_off;        // int64 [n_proj + 1]
    chf::DevBuf sup_row;        // int32 [pairs]
    chf::DevBuf ent_off;        // int64 [n_rows + 1]
    chf::DevBuf ent_off32;      // int32 [n_rows + 1] (pairs < 2^31)
    chf::DevBuf ent_atom;       // int32 [pairs]
    chf::DevBuf ent_soff;       // int32 [pairs] LDS byte offset of that slot's staged coefficients (slot * 512)
    chf::DevBuf quad_count;     // uint64 [n_blocks][16]: byte z = largest entry count of the wave's
                                //   4 rows (quad) in plane z, capped at 255
    chf::DevBuf blk_atom_off;   // int32 [n_blocks + 1]
    chf::DevBuf blk_atoms;      // int32 [sum of block atom counts]
    chf::DevBuf sup_beta64, ent_beta64;  // double [pairs][4]
    chf::DevBuf sup_beta32, ent_beta32;  // float  [pairs][4]
    chf::DevBuf kb_coef;        // KB coefficients scratch [4 n_proj][nvec] in the work dtype
    chf::DevBuf flag;           // int: set by the V_eff cast when a value is NaN or Inf
    int dtypes = 0;
    bool has_nbr = false;
    // Poisson exterior stencil points (built on first use, scf.hip)
    chf::DevBuf ghost_owner;    // int32 [n_ghost] row of the inside point
    chf::DevBuf ghost_k;        // int32 [n_ghost] |offset| 1..6
    chf::DevBuf ghost_ijk;      // int32 [n_ghost][3]
    int64_t n_ghost = -1;
    hipStream_t stream = nullptr;  // stream of the last call (for destroy)
};

// bytes of chf_ctx::info, allocated with the context: a few device scalars
// (reduction results, factorisation status) and up to 32 Anderson
// coefficients
constexpr size_t kInfoBytes = 4096;

struct chf_ctx {
    int device = 0;
    rocblas_handle blas = nullptr;
    chf::DevBuf scratch;        // M x M FP64 and split-K partials
    chf::DevBuf scratch2;
    chf::DevBuf info;           // int device scalars
    chf::DevBuf vec;            // FP64 vectors for Lanczos / CG
    chf::DevBuf red;            // reduction partials
};
