// Internal declarations shared by the HIP kernels and the C-ABI runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ocean_bse.h"

namespace ocean {

constexpr int kMaxCore = 12;    // Nc limit of the combine and local kernels (12: 2p with electron spin)
constexpr int kMaxLocal = 64;   // Nmu limit (4 radial functions x 16 lm of s, p, d, f)
constexpr int kMaxPairs = 768;  // Nc * Nmu limit of the local kernels (12 x 64)
constexpr int kMaxDft = 16;     // largest k-grid extent per axis
constexpr int kColsPerPass = 24;  // exciton columns per projection launch (3 MFMA column tiles)
constexpr int kColsPerWidePass = 40;  // FP64 single pass for 25..40 columns (5 column tiles)
constexpr int kRedBlocks = 240;   // blocks per vector in the Lanczos reductions
constexpr int kXB = 16;           // x-block of the phi work array (a power of two: phi_index_x)
constexpr int kStageTile = 4096;
constexpr int kCombineDirectChunks = 4;  // up to this many x chunks the combine pass sums the
                                          // back-projection partials itself  // bytes of one staged B chunk per 16-wide column tile

// phi work array layout: [x / kXB][k][x % kXB][col] (complex).  A "line" is
// line = x * cols + col; for a fixed k the lines of one x-block are contiguous,
// so the k-grid transform touches one contiguous region per x-block.
__host__ __device__ inline size_t phi_index(long long line, int k, int Nk, int cols) {
    const long long xbc = (long long)kXB * cols;
    const long long xb = line / xbc;
    return (size_t)((xb * Nk + k) * xbc + (line - xb * xbc));
}

// Same index from the point x and column col (no division: kXB is a power of two).
__host__ __device__ inline size_t phi_index_x(int x, int col, int k, int Nk, int cols) {
    return ((size_t)((x >> 4) * Nk + k) * kXB + (x & (kXB - 1))) * cols + col;
}

// Bytes of the phi work array of a pass with `cols` columns (x padded to whole x-blocks),
// the extent of a buffer descriptor over it.
__host__ __device__ inline size_t phi_span_bytes(int Nx, int Nk, int cols, int elem) {
    return (size_t)((Nx + kXB - 1) / kXB) * kXB * Nk * cols * elem;
}

// Per-vector Lanczos state kept on the device.
struct LzState {
    double b_cur;   // b_i of the current step (b_0 = 0)
    double scale;   // running max(|a_0..a_i|, b_1..b_i)
    double norm2;   // |psi0|^2
    double a_cur;
    int done;       // 1 once the recursion has stopped for this vector
    int steps;      // completed steps
    int pad[2];
};

// Workspace of one H*v for up to `cols` exciton columns.
struct Workspace {
    int cols = 0;
    int bwd_chunks = 0;
    void* phi = nullptr;        // [Nk][Nx][cols] complex (FP64 or FP32)
    double* part = nullptr;     // [S][Nk][Nb][cols] complex back-projection partials
    double* w0 = nullptr;       // [Nk][Nb][cols] complex: the partials summed (W0 x)
    double* loc_part = nullptr; // [P][nv][Nc*Nmu] complex
    double* loc_b = nullptr;    // [nv][Nc*Nmu] complex
    unsigned char* bst = nullptr;  // bf16 modes: forward B operand of one projection pass,
                                   // staged per (k, band chunk) in the kernel's LDS order
    size_t bytes = 0;
};

struct LanczosBuffers {
    int nv = 0, n_steps = 0;
    bool reorth = false;
    double* v = nullptr;       // [nv][dim] complex
    double* vprev = nullptr;
    double* w = nullptr;
    double* basis = nullptr;   // [nv][n_steps+1][dim] complex (reorth only)
    double* part_a = nullptr;  // [nv][kRedBlocks]
    double* part_n = nullptr;
    double* hpart = nullptr;   // [nv][kRedBlocks][n_steps+1] complex (reorth only)
    double* hcoef = nullptr;   // [nv][n_steps+1] complex (reorth only)
    double* a = nullptr;       // [nv][n_steps]
    double* b = nullptr;
    LzState* state = nullptr;  // [nv]
    int* step = nullptr;
    size_t bytes = 0;
};

struct KernelStat {
    const char* name;
    double ms;
    long long count;
};

}  // namespace ocean

struct ocean_bse_s {
    int nk[3], nx[3];
    int Nk, Nx, Nb, Nc, Nmu;
    double cell[9], tau[3];      // lattice vectors as rows (a1, a2, a3), bohr
    int precision;
    unsigned flags;
    int device;
    hipStream_t stream;
    bool own_stream;

    // inputs resident on the device
    double* E = nullptr;            // [Nk][Nb]
    const double* U64 = nullptr;    // [Nk][Nx][Nb] complex (owned or borrowed)
    double* U64_owned = nullptr;
    // true when the stored u (every owned copy: FP64, FP32, bf16) already carries the Bloch
    // phase e^{ik.x}, so that the k-grid transform has no phase to apply; false for a
    // borrowed FP64 array, which is used as given
    bool u_phased = false;
    float* U32 = nullptr;           // [Nk][Nx][Nb] complex FP32 copy (FP32 mode)
    uint16_t* Ubf = nullptr;        // bf16 modes: hi plane [Nk][Nx][Nb][re, im], then (split) the residual plane
    uint16_t* UbfT = nullptr;       // the same values transposed, [Nk][Nb][NxP][re, im] (+ residual plane),
                                    // rows padded with zeros to NxP = Nx rounded up to 4; read by the
                                    // back-projection so that 4 consecutive x are one 16-byte load
    int NxP = 0;
    double* W64 = nullptr;          // [Nx][R2 R3][R1] W(x, R) / Nk
    float* W32 = nullptr;
    double* phase = nullptr;        // per-axis e^{2 pi i a b / (n g)} tables, complex
    double* twiddle = nullptr;      // per-axis e^{2 pi i m / n} tables, complex
    int phase_off[3], tw_off[3];
    double* A = nullptr;            // [Nk][Nb][Nmu] complex
    double* K = nullptr;            // [(Nc Nmu)^2] complex
    double* Hc = nullptr;           // [Nc^2] complex

    ocean::Workspace ws;
    ocean::LanczosBuffers lz;

    // tuning knobs (picked at create, overridable through the environment)
    int fft_lines = 16;          // lines per block of the k-grid transform
    int fft_pairs = 1;           // FP32-arithmetic cube transform: two lines per thread
    int bwd_target_blocks = 2048;  // back-projection grid size the x chunking aims at
    int bwd_waves = 8;           // back-projection: at most this many waves (16 bands each) per block
    int fwd_ms = 2;              // forward projection: 16 * fwd_ms rows per wave
    int quad_tail = 1;           // FP32: a remainder of <= 4 real columns on the 4x4x1 MFMA (0: a padded tile)
    int fwd_tiles = 0;           // FP64/FP32 forward with psi[k] resident in LDS: row tiles per block
                                 // (0: the band-chunked kernel; used only where psi[k] fits)

    // profiling
    bool profiling = false;
    std::vector<ocean::KernelStat> stats;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;

    size_t device_bytes = 0;
};

namespace ocean {

// Raw buffer access: loads at offsets beyond the descriptor extent return zero and stores
// there are dropped, which replaces bounds branches in the streaming kernels.
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr unsigned kOob = 0xFFFFFFF0u;  // an offset beyond every descriptor extent

__device__ __forceinline__ Rsrc make_rsrc(const void* base, size_t bytes) {
    const unsigned n = bytes >= 0xFFFFFFF0ull ? 0xFFFFFFF0u : (unsigned)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)n, 0x00020000);
}
template <typename C2> __device__ __forceinline__ C2 bload(Rsrc r, unsigned off);
template <> __device__ __forceinline__ double2 bload<double2>(Rsrc r, unsigned off) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}
template <> __device__ __forceinline__ float2 bload<float2>(Rsrc r, unsigned off) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
// Loads of a stream read once in whole 128-byte lines (u in the back-projections): the
// non-temporal cache policy (cache-policy bit 1, "nt" on gfx950), so the stream does not
// displace reused lines.  The forward projections read each line of u in two 64-byte halves
// by consecutive instructions and rely on the second half hitting in the cache; with this
// policy the FP64 forward was 10% slower, the back-projection 2% faster.
constexpr int kStreamPolicy = 2;
template <typename C2> __device__ __forceinline__ C2 bload_stream(Rsrc r, unsigned off);
template <> __device__ __forceinline__ double2 bload_stream<double2>(Rsrc r, unsigned off) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, kStreamPolicy));
}
template <> __device__ __forceinline__ float2 bload_stream<float2>(Rsrc r, unsigned off) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, kStreamPolicy));
}
// The projections' intermediate phi in the BF16 mode: a complex value stored as two bf16
// (4 bytes).  Loads widen to float2, stores round to nearest even.  In the other modes phi is
// stored in its compute type and these are plain accesses.
struct alignas(4) bf16c {
    __bf16 x, y;
};
template <typename C2, typename S> __device__ __forceinline__ C2 phi_load(const S* p) { return *p; }
template <> __device__ __forceinline__ float2 phi_load<float2, bf16c>(const bf16c* p) {
    const bf16c v = *p;
    return make_float2((float)v.x, (float)v.y);
}
template <typename C2, typename S> __device__ __forceinline__ void phi_store(S* p, C2 v) { *p = v; }
template <> __device__ __forceinline__ void phi_store<float2, bf16c>(bf16c* p, float2 v) {
    bf16c s;
    s.x = (__bf16)v.x;
    s.y = (__bf16)v.y;
    *p = s;
}
// bytes of one stored phi element
inline size_t phi_elem_bytes(int precision) {
    return precision == OCEAN_PREC_FP64 ? 16 : precision == OCEAN_PREC_BF16 ? 4 : 8;
}

template <typename C2> __device__ __forceinline__ void bstore(C2 v, Rsrc r, unsigned off);
template <> __device__ __forceinline__ void bstore<double2>(double2 v, Rsrc r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), r, (int)off, 0, 0);
}
template <> __device__ __forceinline__ void bstore<float2>(float2 v, Rsrc r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r, (int)off, 0, 0);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4v __attribute__((ext_vector_type(4)));

// Store one 16x16 result tile of the forward projection (register r of lane i + 16 kq:
// row 4 kq + r, real column i of the tile) as two complex columns per lane.  The four lanes
// of a quad transpose their four registers with two exchange rounds, after which lane
// 4 a + p holds row 4 kq + p, real columns 4 a .. 4 a + 3 (complex columns 2 a, 2 a + 1 of
// the tile): one store instruction per tile covers it, against four with one real value per
// lane (the store instructions, not the bytes, cost in these kernels).  phi is FP32 pairs
// with LO (the FP32 and split-BF16 modes) and bf16 pairs (rounded to nearest even) without
// (the BF16 mode).  Rows at or
// past Nx and complex columns at or past ncb are not written: a lane whose second column is
// past ncb writes its first one with a narrower store (offsets out of range drop a store).
// pw covers phi from element idx0 on, and every offset written must stay below 4 GiB.
template <bool LO>
__device__ __forceinline__ void store_fwd_tile(f32x4 a, Rsrc pw, size_t idx0, int lane, int rowtop, int c_tile,
                                               int Nx, int ncb, int col0, int k, int Nk, int cols) {
    const int i = lane & 15, kq = lane >> 4, p = i & 3;
    float v[4] = {a[0], a[1], a[2], a[3]};
#pragma unroll
    for (int b = 1; b <= 2; b <<= 1) {
#pragma unroll
        for (int r0 = 0; r0 < 4; ++r0) {
            if (r0 & b) continue;
            const int r1 = r0 | b;
            const bool hi = p & b;
            const float t = __shfl_xor(hi ? v[r0] : v[r1], b);
            if (hi) v[r0] = t;
            else v[r1] = t;
        }
    }
    const int row = rowtop + 4 * kq + p;
    const int c = c_tile + 2 * (i >> 2);
    const bool rok = row < Nx;
    const unsigned base = (unsigned)(phi_index_x(row, col0 + c, k, Nk, cols) - idx0) * (LO ? 8u : 4u);
    const unsigned off2 = (rok && c + 1 < ncb) ? base : kOob;
    const unsigned off1 = (rok && c + 1 == ncb) ? base : kOob;
    if constexpr (LO) {
        typedef float f2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4v, f32x4{v[0], v[1], v[2], v[3]}), pw, (int)off2, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, f2{v[0], v[1]}),
                                              pw, (int)off1, 0, 0);
    } else {
        const bf16c c0{(__bf16)v[0], (__bf16)v[1]}, c1{(__bf16)v[2], (__bf16)v[3]};
        const unsigned w0 = __builtin_bit_cast(unsigned, c0), w1 = __builtin_bit_cast(unsigned, c1);
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(u2{w0, w1}, pw, (int)off2, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b32(w0, pw, (int)off1, 0, 0);
    }
}

// Bloch phase e^{ik.x} of row g = k Nx + x of u, from the per-axis tables
// ph[po[a] + i n_x[a]... ] = e^{2 pi i i_a j_a / (n_k[a] n_x[a])}.
// Geometry of the W(x, R) table: cell rows A, supercell rows S = n_d a_d and S^-1 (row-major,
// row-vector convention: cartesian = fractional . rows), tau, and whether the S_d are
// mutually orthogonal (then the wrapped image is the nearest).
struct WGeom {
    double A[9], S[9], Sinv[9], tau[3];
    int ortho;
};

struct PhaseArgs {
    const double* ph;
    int po[3], nk[3], nx[3];
    long long Nx;
};

__device__ inline double2 bloch_phase(const PhaseArgs& p, long long g) {
    const long long k = g / p.Nx;
    const long long x = g - k * p.Nx;
    const int i3 = (int)(k % p.nk[2]), i2 = (int)((k / p.nk[2]) % p.nk[1]), i1 = (int)(k / ((long long)p.nk[1] * p.nk[2]));
    const int j3 = (int)(x % p.nx[2]), j2 = (int)((x / p.nx[2]) % p.nx[1]), j1 = (int)(x / ((long long)p.nx[1] * p.nx[2]));
    const double2* t = reinterpret_cast<const double2*>(p.ph);
    const double2 a = t[p.po[0] + i1 * p.nx[0] + j1], b = t[p.po[1] + i2 * p.nx[1] + j2], c = t[p.po[2] + i3 * p.nx[2] + j3];
    const double2 ab = make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
    return make_double2(ab.x * c.x - ab.y * c.y, ab.x * c.y + ab.y * c.x);
}

void set_error(const std::string& msg);
size_t max_device_bytes();

// Kernel launchers (each enqueues on h->stream).  Return hipSuccess or the launch error.
hipError_t launch_proj_fwd(ocean_bse_s* h, const double* x, int nv, int col0, int ncb);
int fwd_band_chunk(const ocean_bse_s* h);  // bands per staged forward chunk, 0 if not staged
bool is_bf16_mode(int precision);
hipError_t launch_proj_fwd_bf16(ocean_bse_s* h, const double* x, int nv, int col0, int ncb);
hipError_t launch_proj_bwd_bf16(ocean_bse_s* h, int nv, int col0, int ncb);
hipError_t launch_fft_w(ocean_bse_s* h, int cols);
hipError_t launch_proj_bwd(ocean_bse_s* h, int nv, int col0, int ncb);
hipError_t launch_local_in(ocean_bse_s* h, const double* x, int nv);
hipError_t launch_local_mat(ocean_bse_s* h, int nv);
hipError_t launch_combine(ocean_bse_s* h, const double* x, double* y, int nv, double* dot_part);
hipError_t launch_reduce_part(ocean_bse_s* h, int nv);
hipError_t launch_w_gamma(ocean_bse_s* h, int cols);
hipError_t launch_build_w(ocean_bse_s* h, const double* wr_dev, const double* wv_dev, int n_wr,
                          double h_r);
// u rows g0 .. g0 + rows - 1 (FP64, at src) times their Bloch phase, stored in the handle's
// precision: FP64 in place (src may equal dst), FP32, or the bf16 planes of both layouts
PhaseArgs phase_args(const ocean_bse_s* h);
hipError_t launch_u_phase_fp64(ocean_bse_s* h, const double* src, long long g0, long long rows, double* dst);
hipError_t launch_u_to_fp32(ocean_bse_s* h, const double* src, long long g0, long long rows, float* dst);
hipError_t launch_u_to_bf16(ocean_bse_s* h, const double* src, long long g0, long long rows);
hipError_t launch_dipole_psi0(ocean_bse_s* h, const double* d_dev, int n_pol, double* psi0);

// Lanczos kernels
hipError_t lz_init(ocean_bse_s* h, const double* psi0, int nv);
hipError_t lz_dot_vw(ocean_bse_s* h, int nv);
hipError_t lz_update(ocean_bse_s* h, int nv, bool with_norm);
hipError_t lz_reorth(ocean_bse_s* h, int nv);
hipError_t lz_norm_w(ocean_bse_s* h, int nv);
hipError_t lz_finalize(ocean_bse_s* h, int nv);
hipError_t lz_scale(ocean_bse_s* h, int nv);
hipError_t lz_advance(ocean_bse_s* h);

hipError_t launch_spectrum(const double* a, const double* b, const int* n_used, const double* norm2,
                           int n_spec, int n_steps, int terminator, const double* a_inf,
                           const double* b_inf, const double* omega,
                           int n_omega, double gamma, double* sigma, hipStream_t stream);

// geometry helpers
int bwd_waves_for(int Nb, int cap);
int bwd_waves(const ocean_bse_s* h);
int cols_per_pass(const ocean_bse_s* h, int cols);
void bwd_geometry(const ocean_bse_s* h, int* band_blocks, int* S, int* chunk);
void bwd_geometry_for(const ocean_bse_s* h, int target_blocks, int W, int* band_blocks, int* S, int* chunk);
constexpr int kMaxBwdTarget = 8192;  // largest back-projection grid target the tuner tries
size_t fft_lds_bytes(const ocean_bse_s* h, int lines);
size_t fwd_res_lds_bytes(const ocean_bse_s* h, int ncb);   // 0: psi[k] does not fit
long long local_blocks(const ocean_bse_s* h);

// profiling helpers used by the launchers
int prof_begin(ocean_bse_s* h, const char* name);
void prof_end(ocean_bse_s* h, int slot);

}  // namespace ocean
