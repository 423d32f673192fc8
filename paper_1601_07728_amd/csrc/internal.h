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

constexpr int kMaxCore = 8;     // Nc limit of the combine kernel
constexpr int kMaxLocal = 16;   // Nmu limit
constexpr int kMaxPairs = 128;  // Nc * Nmu limit of the local kernels
constexpr int kMaxDft = 16;     // largest k-grid extent per axis
constexpr int kColsPerPass = 24;  // exciton columns per projection launch (3 MFMA column tiles)
constexpr int kRedBlocks = 240;   // blocks per vector in the Lanczos reductions
constexpr int kXB = 16;           // x-block of the phi work array (a power of two: phi_index_x)

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
    double cell[3], tau[3];
    int precision;
    unsigned flags;
    int device;
    hipStream_t stream;
    bool own_stream;

    // inputs resident on the device
    double* E = nullptr;            // [Nk][Nb]
    const double* U64 = nullptr;    // [Nk][Nx][Nb] complex (owned or borrowed)
    double* U64_owned = nullptr;
    float* U32 = nullptr;           // [Nk][Nx][Nb] complex FP32 copy (FP32 mode)
    uint16_t* Ubf = nullptr;        // bf16 modes: hi plane [Nk][Nx][Nb][re, im], then (split) the residual plane
    uint16_t* UbfT = nullptr;       // the same values transposed, [Nk][Nb][NxP][re, im] (+ residual plane),
                                    // rows padded with zeros to NxP = Nx rounded up to 4; read by the
                                    // back-projection so that 4 consecutive x are one 16-byte load
    int NxP = 0;
    double* W64 = nullptr;          // [Nx][Nk] W(x, R)
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
    int bwd_target_blocks = 2048;  // back-projection grid size the x chunking aims at
    int fwd_ms = 2;              // forward projection: 16 * fwd_ms rows per wave

    // profiling
    bool profiling = false;
    std::vector<ocean::KernelStat> stats;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;

    size_t device_bytes = 0;
};

namespace ocean {

void set_error(const std::string& msg);
size_t max_device_bytes();

// Kernel launchers (each enqueues on h->stream).  Return hipSuccess or the launch error.
hipError_t launch_proj_fwd(ocean_bse_s* h, const double* x, int nv, int col0, int ncb);
hipError_t launch_fft_w(ocean_bse_s* h, int cols);
hipError_t launch_proj_bwd(ocean_bse_s* h, int nv, int col0, int ncb);
hipError_t launch_local_in(ocean_bse_s* h, const double* x, int nv);
hipError_t launch_local_mat(ocean_bse_s* h, int nv);
hipError_t launch_combine(ocean_bse_s* h, const double* x, double* y, int nv, double* dot_part);
hipError_t launch_reduce_part(ocean_bse_s* h, int nv);
hipError_t launch_w_gamma(ocean_bse_s* h, int cols);
hipError_t launch_build_w(ocean_bse_s* h, const double* wr_dev, const double* wv_dev, int n_wr,
                          double h_r);
hipError_t launch_to_fp32(ocean_bse_s* h, const double* src, float* dst, long long n);
hipError_t launch_to_bf16(ocean_bse_s* h, const double* src, uint16_t* hi, uint16_t* lo, long long n);
hipError_t launch_to_bf16_t(ocean_bse_s* h, const double* src, long long g0, long long rows, uint16_t* hiT,
                            uint16_t* loT);
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
                           int n_spec, int n_steps, int terminator, const double* omega,
                           int n_omega, double gamma, double* sigma, hipStream_t stream);

// geometry helpers
int bwd_waves(int Nb);
void bwd_geometry(const ocean_bse_s* h, int* band_blocks, int* S, int* chunk);
void bwd_geometry_for(const ocean_bse_s* h, int target_blocks, int* band_blocks, int* S, int* chunk);
constexpr int kMaxBwdTarget = 8192;  // largest back-projection grid target the tuner tries
size_t fft_lds_bytes(const ocean_bse_s* h, int lines);
long long local_blocks(const ocean_bse_s* h);

// profiling helpers used by the launchers
int prof_begin(ocean_bse_s* h, const char* name);
void prof_end(ocean_bse_s* h, int slot);

}  // namespace ocean
