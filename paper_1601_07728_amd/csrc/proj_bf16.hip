// Band projections of Algorithm 1 (section 3.2.1) on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation): the split-BF16 and BF16 precision modes.
// The contractions and their real-GEMM form are those of proj.hip.  u~ is stored as a bf16
// hi plane and, in the split mode, a plane holding the rounding residual; the B operand (psi
// forward, phi' back) is split into hi + residual when it is staged, and the products
// hi*hi + hi*lo (+ lo*hi in the split mode) are accumulated, so the operand rounding of the
// dominant terms is compensated.
//
// A sub-step covers 16 contraction points: lane l = i + 16 kq holds points 4 kq .. 4 kq + 3,
// slot 2 m + p = part p of point m; result register r holds column i of row 4 kq + r.
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace ocean {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

__device__ __forceinline__ v4f mfma_bf16(bf16x8 a, bf16x8 b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}


// v = hi + lo with hi = v rounded to bf16 and lo the rounded residual
__device__ __forceinline__ void split_d(double v, __bf16& hi, __bf16& lo) {
    hi = (__bf16)(float)v;
    lo = (__bf16)(float)(v - (double)(float)hi);
}
__device__ __forceinline__ void split_f(float v, __bf16& hi, __bf16& lo) {
    hi = (__bf16)v;
    lo = (__bf16)(v - (float)hi);  // exact in FP32
}

// Workgroups are dealt round-robin to the 8 XCDs; this renumbering gives each XCD a
// contiguous run of blocks, so the blocks that share a k (and its staged B operand) meet in
// one L2.
__device__ __forceinline__ int xcd_block() {
    const unsigned nblk = gridDim.x, q8 = nblk / 8, r8 = nblk % 8;
    const unsigned xcd = blockIdx.x % 8, pos = blockIdx.x / 8;
    return (int)(xcd * q8 + (xcd < r8 ? xcd : r8) + pos);
}

// Wait until at most N vector-memory loads of this wave are outstanding (vmcnt counts loads
// in issue order); expcnt and lgkmcnt are left alone.
template <int N> __device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// Copy staged chunk ch (CB = NT * 4 KiB bytes) straight from memory into an LDS buffer:
// buffer_load ... lds writes lane l's 16 bytes at the wave's LDS base + 16 l, so the 256
// threads move the chunk in NT rounds of 4 KiB with no registers in between.  Offsets past
// the last chunk are outside the descriptor and read zero.
template <int NT>
__device__ __forceinline__ void copy_chunk_lds(Rsrc br, void* lds_buf, int ch) {
    constexpr int CB = NT * kStageTile;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NT; ++j)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            br, (__attribute__((address_space(3))) void*)(static_cast<unsigned char*>(lds_buf) + (j * 256 + 64 * wave) * 16),
            16, (int)((unsigned)ch * CB + (j * 256 + threadIdx.x) * 16u), 0, 0, 0);
}

// ---------------------------------------------------------------------------------------------
// Forward B operand of the bf16 kernels, staged once per apply.  Every x tile of a k uses the
// same psi chunk, so the chunk is split into bf16 hi + residual and laid out here, in exactly
// the byte order of the kernel's LDS buffer, for all (k, band chunk): the projection kernel
// then only copies 16-byte pieces.  One item = one (k, chunk, sub-step, column tile, lane);
// padding columns and bands are zero.
// chunk = [hi plane][lo plane], each [ss][t][lane][8] with 16-point sub-steps
__global__ __launch_bounds__(256) void prep_fwd_b_bf16_kernel(const double2* __restrict__ psi,
                                                             unsigned char* __restrict__ out, int Nk, int Nb,
                                                             int Nc, int col0, int ncb, int NT, int nchunks) {
    constexpr int KC = 32, SS = KC / 16;
    const int BUF = SS * NT * 64 * 8;  // bf16 values per plane
    const long long total = (long long)Nk * nchunks * SS * NT * 64;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int lane = (int)(e & 63);
        long long r = e >> 6;
        const int t = (int)(r % NT);
        r /= NT;
        const int ss = (int)(r % SS);
        r /= SS;
        const int ch = (int)(r % nchunks);
        const int k = (int)(r / nchunks);
        const int i = lane & 15, kq = lane >> 4;
        const int jr = 16 * t + i, cl = jr >> 1, q = jr & 1;
        bf16x8 hv, lv;
#pragma unroll
        for (int j = 0; j < 8; ++j) hv[j] = lv[j] = (__bf16)0.f;
        if (cl < ncb) {
            const int col = col0 + cl, vv = col / Nc, c = col - vv * Nc;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int n = ch * KC + 16 * ss + 4 * kq + m;
                if (n < Nb) {
                    const double2 z = psi[(((size_t)vv * Nk + k) * Nb + n) * Nc + c];
                    __bf16 h0, l0, h1, l1;
                    split_d(q ? z.y : z.x, h0, l0);
                    split_d(q ? z.x : -z.y, h1, l1);
                    hv[2 * m] = h0;
                    lv[2 * m] = l0;
                    hv[2 * m + 1] = h1;
                    lv[2 * m + 1] = l1;
                }
            }
        }
        __bf16* dst = reinterpret_cast<__bf16*>(out + ((size_t)k * nchunks + ch) * NT * kStageTile);
        const int o = ((ss * NT + t) * 64 + lane) * 8;
        *reinterpret_cast<bf16x8*>(dst + o) = hv;
        *reinterpret_cast<bf16x8*>(dst + BUF + o) = lv;
    }
}

template <int MS, int NT, bool LO>
__global__ __launch_bounds__(256) void proj_fwd_bf16_kernel(
    const u16* __restrict__ Uh, const u16* __restrict__ Ul, const unsigned char* __restrict__ bst,
    void* __restrict__ phi, int Nk, int Nx, int Nb, int cols, int col0, int ncb, int x_tiles, int nchunks) {
    constexpr int KC = 32, SS = KC / 16;
    constexpr int BUF = SS * NT * 64 * 8;      // bf16 values per plane
    constexpr int CB = NT * kStageTile;
    static_assert(2 * BUF * 2 == CB, "chunk layout");
    __shared__ __align__(16) __bf16 sB[2][2 * BUF];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const int lblk = xcd_block();
    const int k = lblk / x_tiles;
    const int xt = lblk - k * x_tiles;
    const int rowbase = xt * (64 * MS) + wave * (16 * MS);
    const int brow0 = xt * (64 * MS);
    const int brows = min(Nx - brow0, 64 * MS);
    const size_t plane0 = ((size_t)k * Nx + brow0) * Nb * 2;
    const Rsrc urh = make_rsrc(Uh + plane0, (size_t)brows * Nb * 4);
    const Rsrc url = make_rsrc(LO ? Ul + plane0 : Uh + plane0, (size_t)brows * Nb * 4);
    const Rsrc br = make_rsrc(bst + (size_t)k * nchunks * CB, (size_t)nchunks * CB);
    bool rval[MS];
    unsigned urow[MS];
#pragma unroll
    for (int ms = 0; ms < MS; ++ms) {
        const int row = rowbase + 16 * ms + i;
        rval[ms] = row < Nx;
        urow[ms] = (unsigned)((row - brow0) * Nb) * 4u;
    }
    // A: the four points 4 kq .. 4 kq + 3 of a sub-step are four consecutive bands of row i,
    // one 16-byte load per plane.  A group that straddles Nb reads into the next row (or the
    // zeroed padding after the last plane); those values meet zero B entries.
    auto load_a = [&](int n0, u32x4 (&ah)[MS][SS], u32x4 (&al)[MS][SS]) {
#pragma unroll
        for (int ss = 0; ss < SS; ++ss) {
            const int n = n0 + 16 * ss + 4 * kq;
            const bool nok = n < Nb;
#pragma unroll
            for (int ms = 0; ms < MS; ++ms) {
                const unsigned off = (nok && rval[ms]) ? urow[ms] + (unsigned)n * 4u : kOob;
                ah[ms][ss] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(urh, (int)off, 0, 0));
                if (LO) al[ms][ss] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(url, (int)off, 0, 0));
            }
        }
    };

    v4f acc[MS][NT];
#pragma unroll
    for (int ms = 0; ms < MS; ++ms)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[ms][t] = v4f{0.f, 0.f, 0.f, 0.f};

    u32x4 ah[MS][SS], al[MS][SS], ahn[MS][SS], aln[MS][SS];
    copy_chunk_lds<NT>(br, sB[0], 0);
    load_a(0, ah, al);
    __builtin_amdgcn_s_waitcnt(0);
    int buf = 0;
    for (int n0 = 0, ch = 0; n0 < Nb; n0 += KC, ++ch) {
        __syncthreads();
        // B of the current chunk into registers before the copy into the other buffer
        bf16x8 bh[SS][NT], bl[SS][NT];
#pragma unroll
        for (int ss = 0; ss < SS; ++ss)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                bh[ss][t] = *reinterpret_cast<const bf16x8*>(&sB[buf][((ss * NT + t) * 64 + lane) * 8]);
                bl[ss][t] = *reinterpret_cast<const bf16x8*>(&sB[buf][BUF + ((ss * NT + t) * 64 + lane) * 8]);
            }
        copy_chunk_lds<NT>(br, sB[buf ^ 1], ch + 1);
        __builtin_amdgcn_sched_barrier(0);
        load_a(n0 + KC, ahn, aln);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ss = 0; ss < SS; ++ss) {
#pragma unroll
            for (int ms = 0; ms < MS; ++ms) {
                const bf16x8 a_h = __builtin_bit_cast(bf16x8, ah[ms][ss]);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    acc[ms][t] = mfma_bf16(a_h, bh[ss][t], acc[ms][t]);
                    acc[ms][t] = mfma_bf16(a_h, bl[ss][t], acc[ms][t]);
                }
                if (LO) {
                    const bf16x8 a_l = __builtin_bit_cast(bf16x8, al[ms][ss]);
#pragma unroll
                    for (int t = 0; t < NT; ++t) acc[ms][t] = mfma_bf16(a_l, bh[ss][t], acc[ms][t]);
                }
            }
        }
        wait_vmcnt<MS * SS * (LO ? 2 : 1)>();
#pragma unroll
        for (int ms = 0; ms < MS; ++ms)
#pragma unroll
            for (int ss = 0; ss < SS; ++ss) {
                ah[ms][ss] = ahn[ms][ss];
                if (LO) al[ms][ss] = aln[ms][ss];
            }
        buf ^= 1;
    }

    // phi: FP32 pairs in the split mode, bf16 pairs in the BF16 mode (store_fwd_tile)
    constexpr int E = LO ? 8 : 4;
    const size_t idx0 = phi_index_x(xt * (64 * MS), col0, k, Nk, cols);
    const Rsrc pw = make_rsrc(static_cast<unsigned char*>(phi) + idx0 * E, phi_span_bytes(Nx, Nk, cols, E) - idx0 * E);
#pragma unroll
    for (int ms = 0; ms < MS; ++ms)
#pragma unroll
        for (int t = 0; t < NT; ++t)
            store_fwd_tile<LO>(acc[ms][t], pw, idx0, lane, rowbase + 16 * ms, 8 * t, Nx, ncb, col0, k, Nk, cols);
}

// Forward with the staged B operand resident.  When the B chunks of psi[k] for every band
// fit in LDS (96 bands and three column tiles: 3 chunks of 12 KiB), a block copies them once
// and then streams u for `tiles` consecutive tiles of 64 MS rows of that k.  Each wave owns
// 16 MS rows of every tile and walks its (tile, band chunk) items as one continuous pipeline:
// the u loads of the next item (the next chunk, or the first chunk of the next tile) are in
// flight while the current one is contracted, and there is no barrier after the staging.
// The MFMA sequence of every output element is the chunked kernel's.
template <int MS, int NT, bool LO>
__global__ __launch_bounds__(256) void proj_fwd_bf16_res_kernel(
    const u16* __restrict__ Uh, const u16* __restrict__ Ul, const unsigned char* __restrict__ bst,
    void* __restrict__ phi, int Nk, int Nx, int Nb, int cols, int col0, int ncb, int x_tiles, int nchunks,
    int groups, int tiles) {
    constexpr int KC = 32, SS = KC / 16;
    constexpr int BUF = SS * NT * 64 * 8;      // bf16 values per plane of one chunk
    constexpr int CB = NT * kStageTile;        // bytes of one staged chunk (both planes)
    static_assert(2 * BUF * 2 == CB, "chunk layout");
    extern __shared__ __align__(16) unsigned char smem[];   // [nchunks][CB]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const int lblk = xcd_block();
    const int k = lblk / groups;
    const int g = lblk - k * groups;
    const int t0 = g * tiles, t1 = min(x_tiles, t0 + tiles);
    if (t0 >= t1) return;   // the whole block, before any barrier
    // u planes of this k (offsets fit 32 bits: the launcher requires Nx Nb 4 < 2^31)
    const size_t plane0 = (size_t)k * Nx * Nb * 2;
    const Rsrc urh = make_rsrc(Uh + plane0, (size_t)Nx * Nb * 4);
    const Rsrc url = make_rsrc(LO ? Ul + plane0 : Uh + plane0, (size_t)Nx * Nb * 4);
    const Rsrc br = make_rsrc(bst + (size_t)k * nchunks * CB, (size_t)nchunks * CB);
    for (int ch = 0; ch < nchunks; ++ch) copy_chunk_lds<NT>(br, smem + (size_t)ch * CB, ch);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // A of item (tile, chunk): as in the chunked kernel, the four points 4 kq .. 4 kq + 3 of a
    // sub-step are four consecutive bands of row i, one 16-byte load per plane (a group that
    // straddles Nb reads into the next row or past the plane, where B is zero); masked to zero
    // past Nx or when !live
    auto load_a = [&](int tile, int ch, bool live, u32x4 (&ah)[MS][SS], u32x4 (&al)[MS][SS]) {
        const int rowbase = tile * (64 * MS) + wave * (16 * MS);
#pragma unroll
        for (int ss = 0; ss < SS; ++ss) {
            const int n = ch * KC + 16 * ss + 4 * kq;
            const bool nok = live && n < Nb;
#pragma unroll
            for (int ms = 0; ms < MS; ++ms) {
                const int row = rowbase + 16 * ms + i;
                const unsigned off = (nok && row < Nx) ? ((unsigned)row * (unsigned)Nb + (unsigned)n) * 4u : kOob;
                ah[ms][ss] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(urh, (int)off, 0, 0));
                if (LO) al[ms][ss] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(url, (int)off, 0, 0));
            }
        }
    };

    v4f acc[MS][NT];
#pragma unroll
    for (int ms = 0; ms < MS; ++ms)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[ms][t] = v4f{0.f, 0.f, 0.f, 0.f};
    auto contract = [&](const u32x4 (&ah)[MS][SS], const u32x4 (&al)[MS][SS], int ch) {
        const __bf16* sb = reinterpret_cast<const __bf16*>(smem + (size_t)ch * CB);
#pragma unroll
        for (int ss = 0; ss < SS; ++ss) {
            bf16x8 bh[NT], bl[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                bh[t] = *reinterpret_cast<const bf16x8*>(&sb[((ss * NT + t) * 64 + lane) * 8]);
                bl[t] = *reinterpret_cast<const bf16x8*>(&sb[BUF + ((ss * NT + t) * 64 + lane) * 8]);
            }
#pragma unroll
            for (int ms = 0; ms < MS; ++ms) {
                const bf16x8 a_h = __builtin_bit_cast(bf16x8, ah[ms][ss]);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    acc[ms][t] = mfma_bf16(a_h, bh[t], acc[ms][t]);
                    acc[ms][t] = mfma_bf16(a_h, bl[t], acc[ms][t]);
                }
                if (LO) {
                    const bf16x8 a_l = __builtin_bit_cast(bf16x8, al[ms][ss]);
#pragma unroll
                    for (int t = 0; t < NT; ++t) acc[ms][t] = mfma_bf16(a_l, bh[t], acc[ms][t]);
                }
            }
        }
    };
    // tile done: write its rows of phi (FP32 pairs in the split mode, bf16 pairs in the BF16
    // mode; store_fwd_tile) and start the next tile from zero
    constexpr int E = LO ? 8 : 4;
    const size_t idx0 = phi_index_x(t0 * (64 * MS), col0, k, Nk, cols);
    const Rsrc pw = make_rsrc(static_cast<unsigned char*>(phi) + idx0 * E, phi_span_bytes(Nx, Nk, cols, E) - idx0 * E);
    auto finish_tile = [&](int tile) {
        const int rowbase = tile * (64 * MS) + wave * (16 * MS);
#pragma unroll
        for (int ms = 0; ms < MS; ++ms)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                store_fwd_tile<LO>(acc[ms][t], pw, idx0, lane, rowbase + 16 * ms, 8 * t, Nx, ncb, col0, k, Nk, cols);
                acc[ms][t] = v4f{0.f, 0.f, 0.f, 0.f};
            }
    };

    u32x4 ah[MS][SS], al[MS][SS], ahn[MS][SS], aln[MS][SS];
    int tile = t0, ch = 0;
    load_a(tile, ch, true, ah, al);
    for (;;) {
        int ntile = tile, nchk = ch + 1;
        if (nchk == nchunks) {
            nchk = 0;
            ++ntile;
        }
        const bool more = ntile < t1;
        load_a(ntile, nchk, more, ahn, aln);
        __builtin_amdgcn_sched_barrier(0);
        contract(ah, al, ch);
        if (nchk == 0) finish_tile(tile);
        if (!more) break;
#pragma unroll
        for (int ms = 0; ms < MS; ++ms)
#pragma unroll
            for (int ss = 0; ss < SS; ++ss) {
                ah[ms][ss] = ahn[ms][ss];
                if (LO) al[ms][ss] = aln[ms][ss];
            }
        tile = ntile;
        ch = nchk;
    }
    __builtin_amdgcn_s_waitcnt(0);   // retire the masked loads past the last item before the exit
}

// Staging item = (column cl, lane group kq, sub-step ss): the four points of that lane group
// are loaded once, split into bf16 hi + residual, and written as the 16-byte slots of lanes
// 2 cl and 2 cl + 1 in both planes.
template <int NT, int W, bool LO>
__global__ __launch_bounds__(64 * W) void proj_bwd_bf16_kernel(
    const u16* __restrict__ UTh, const u16* __restrict__ UTl, const void* __restrict__ phi,
    double* __restrict__ part, int Nk, int Nx, int NxP, int Nb, int cols, int col0, int ncb,
    int band_blocks, int S, int chunk) {
    constexpr int XT = 64, SS = XT / 16;
    constexpr int BUF = SS * NT * 64 * 8;
    __shared__ __align__(16) __bf16 sB[2][2 * BUF];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    // XCD-aware numbering: block b runs on XCD b % 8; each XCD takes a contiguous run of
    // (k, x chunk, band block) items, band block fastest, so that the band blocks reading the
    // same phi' tiles run together on one XCD and share them in its L2
    const int total = Nk * band_blocks * S;
    const int per_xcd = (total + 7) / 8;
    const int item = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
    if (item >= total) return;   // the whole block, before any barrier
    const int bb = item % band_blocks;
    const int s = (item / band_blocks) % S;
    const int k = item / (band_blocks * S);
    const int nbase = bb * 16 * W + 16 * wave;
    const int x_begin = s * chunk;
    const int x_end = min(Nx, x_begin + chunk);
    const int n = nbase + i;
    const bool nval = n < Nb;
    // transposed planes [k][n][NxP]: one k plane per resource
    const size_t plane0 = (size_t)k * Nb * NxP * 2;
    const Rsrc urh = make_rsrc(UTh + plane0, (size_t)Nb * NxP * 4);
    const Rsrc url = make_rsrc(LO ? UTl + plane0 : UTh + plane0, (size_t)Nb * NxP * 4);
    const int xb0 = x_begin / kXB;
    const size_t pbase_i = (size_t)xb0 * Nk * kXB * cols;
    // phi' is stored as FP32 pairs in the split mode and as bf16 pairs in the BF16 mode
    constexpr int PE = LO ? 8 : 4;
    const Rsrc prs = make_rsrc(static_cast<const char*>(phi) + pbase_i * PE,
                               (size_t)((x_end - 1) / kXB - xb0 + 1) * Nk * kXB * cols * PE);

    constexpr int NITEM = kColsPerPass * 4 * SS;
    constexpr int PER = (NITEM + 64 * W - 1) / (64 * W);
    auto load_b = [&](int x0, float2 (&bv)[PER][4]) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = threadIdx.x + 64 * W * j;
            const int cl = e % kColsPerPass, rest = e / kColsPerPass;
            const int iq = rest & 3, ss = rest >> 2;
            const bool item = e < NITEM && cl < ncb;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int x = x0 + 16 * ss + 4 * iq + m;
                const bool ok = item && x < x_end;
                const unsigned off = (unsigned)((phi_index_x(x, col0 + cl, k, Nk, cols) - pbase_i) * PE);
                if constexpr (LO) {
                    bv[j][m] = bload<float2>(prs, ok ? off : kOob);
                } else {
                    // (re, im) bf16 at the lower and upper half-words; a bf16 widens by a shift
                    const unsigned w = (unsigned)__builtin_amdgcn_raw_buffer_load_b32(prs, (int)(ok ? off : kOob), 0, 0);
                    bv[j][m] = make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xFFFF0000u));
                }
            }
        }
    };
    auto store_b = [&](int buf, const float2 (&bv)[PER][4]) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = threadIdx.x + 64 * W * j;
            const int cl = e % kColsPerPass, rest = e / kColsPerPass;
            const int iq = rest & 3, ss = rest >> 2;
            if (e >= NITEM || cl >= ncb) continue;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int jr = 2 * cl + q, t = jr >> 4;
                if (t >= NT) continue;
                bf16x8 hv, lv;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    __bf16 h0, l0, h1, l1;
                    split_f(q ? bv[j][m].y : bv[j][m].x, h0, l0);
                    split_f(q ? -bv[j][m].x : bv[j][m].y, h1, l1);
                    hv[2 * m] = h0;
                    lv[2 * m] = l0;
                    hv[2 * m + 1] = h1;
                    lv[2 * m + 1] = l1;
                }
                const int o = ((ss * NT + t) * 64 + (jr & 15) + 16 * iq) * 8;
                *reinterpret_cast<bf16x8*>(&sB[buf][o]) = hv;
                if (LO) *reinterpret_cast<bf16x8*>(&sB[buf][BUF + o]) = lv;   // zero in the BF16 mode
            }
        }
    };
    // A: the four points 4 kq .. 4 kq + 3 of sub-step ss are consecutive x of row n of the
    // transposed plane, one 16-byte load.  x_begin and chunk are multiples of 8, so a group
    // never crosses a chunk end; past Nx it reads the zero row padding.
    auto load_a = [&](int x0, u32x4 (&ah)[SS], u32x4 (&al)[SS]) {
#pragma unroll
        for (int ss = 0; ss < SS; ++ss) {
            const int x = x0 + 16 * ss + 4 * kq;
            const bool ok = nval && x < x_end;
            const unsigned off = ok ? ((unsigned)n * (unsigned)NxP + (unsigned)x) * 4u : kOob;
            ah[ss] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(urh, (int)off, 0, 0));
            if (LO) al[ss] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(url, (int)off, 0, 0));
        }
    };

    for (int e = threadIdx.x; e < 4 * BUF; e += 64 * W) (&sB[0][0])[e] = (__bf16)0.f;
    v4f acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};

    auto contract = [&](int buf, const u32x4 (&ah)[SS], const u32x4 (&al)[SS]) {
#pragma unroll
        for (int ss = 0; ss < SS; ++ss) {
            const bf16x8 a_h = __builtin_bit_cast(bf16x8, ah[ss]);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const bf16x8 b_h = *reinterpret_cast<const bf16x8*>(&sB[buf][((ss * NT + t) * 64 + lane) * 8]);
                acc[t] = mfma_bf16(a_h, b_h, acc[t]);
                if (LO) {
                    // the FP32 phi' residual (a bf16 phi' has none)
                    const bf16x8 b_l = *reinterpret_cast<const bf16x8*>(&sB[buf][BUF + ((ss * NT + t) * 64 + lane) * 8]);
                    acc[t] = mfma_bf16(a_h, b_l, acc[t]);
                    acc[t] = mfma_bf16(__builtin_bit_cast(bf16x8, al[ss]), b_h, acc[t]);
                }
            }
        }
    };

    // Ring of three tiles: while tile t is contracted, the u and phi' loads of tiles t + 1 and
    // t + 2 are in flight; phi' is staged into LDS one tile ahead (two buffers).  The loop runs
    // whole turns of three tiles (tiles past the chunk end load as zero), so that every step
    // sees the same loads outstanding.
    u32x4 ah[3][SS], al[3][SS];
    float2 bl[3][PER][4];
    load_b(x_begin, bl[0]);
    load_a(x_begin, ah[0], al[0]);
    load_b(x_begin + XT, bl[1]);
    load_a(x_begin + XT, ah[1], al[1]);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    store_b(0, bl[0]);
    int buf = 0;
    auto step = [&](int x0, const u32x4 (&ch)[SS], const u32x4 (&cl)[SS], u32x4 (&nh)[SS], u32x4 (&nl)[SS],
                    float2 (&nb)[PER][4], const float2 (&sb)[PER][4]) {
        __syncthreads();
        load_b(x0 + 2 * XT, nb);
        load_a(x0 + 2 * XT, nh, nl);
        __builtin_amdgcn_sched_barrier(0);
        contract(buf, ch, cl);
        store_b(buf ^ 1, sb);
        buf ^= 1;
    };
    for (int x0 = x_begin; x0 < x_end; x0 += 3 * XT) {
        step(x0, ah[0], al[0], ah[2], al[2], bl[2], bl[1]);
        step(x0 + XT, ah[1], al[1], ah[0], al[0], bl[0], bl[2]);
        step(x0 + 2 * XT, ah[2], al[2], ah[1], al[1], bl[1], bl[0]);
    }
    __builtin_amdgcn_s_waitcnt(0);   // retire the loads past the chunk end before the exit

    double* out = part + ((size_t)s * Nk + k) * Nb * 2 * cols + 2 * col0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int jr = 16 * t + i;
        if ((jr >> 1) >= ncb) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int nn = nbase + 4 * kq + r;
            if (nn < Nb) out[(size_t)nn * 2 * cols + jr] = (double)acc[t][r];
        }
    }
}

// rows g0 .. g0 + rows - 1 of u (row g = k Nx + x, Nb complex FP64 each, starting at src),
// times their Bloch phase, -> bf16 hi (and residual) planes in both layouts: [k][x][n] and
// the transposed [k][n][NxP]
__global__ __launch_bounds__(256) void u_to_bf16_kernel(const double* __restrict__ src, long long g0, long long rows,
                                                       int Nx, int Nb, int NxP, PhaseArgs pa,
                                                       __bf16* __restrict__ hi, __bf16* __restrict__ lo,
                                                       __bf16* __restrict__ hiT, __bf16* __restrict__ loT) {
    const long long n_el = rows * Nb;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n_el; e += stride) {
        const long long r = e / Nb;
        const int n = (int)(e - r * Nb);
        const long long g = g0 + r;
        const double2 ph = bloch_phase(pa, g);
        const double re = src[2 * e], im = src[2 * e + 1];
        const double vr = re * ph.x - im * ph.y, vi = re * ph.y + im * ph.x;
        __bf16 h0, l0, h1, l1;
        split_d(vr, h0, l0);
        split_d(vi, h1, l1);
        const size_t o = 2 * ((size_t)g * Nb + n);
        const long long k = g / Nx;
        const int x = (int)(g - k * Nx);
        const size_t ot = 2 * (((size_t)k * Nb + n) * NxP + x);
        hi[o] = h0;
        hi[o + 1] = h1;
        hiT[ot] = h0;
        hiT[ot + 1] = h1;
        if (lo) {
            lo[o] = l0;
            lo[o + 1] = l1;
            loT[ot] = l0;
            loT[ot + 1] = l1;
        }
    }
}

template <int MS, bool LO>
hipError_t fwd_bf16_nt(int NT, dim3 grid, hipStream_t st, const u16* uh, const u16* ul, const unsigned char* bst,
                       void* phi, int Nk, int Nx, int Nb, int cols, int col0, int ncb, int x_tiles, int nchunks) {
    switch (NT) {
        case 1: proj_fwd_bf16_kernel<MS, 1, LO><<<grid, 256, 0, st>>>(uh, ul, bst, phi, Nk, Nx, Nb, cols, col0, ncb, x_tiles, nchunks); break;
        case 2: proj_fwd_bf16_kernel<MS, 2, LO><<<grid, 256, 0, st>>>(uh, ul, bst, phi, Nk, Nx, Nb, cols, col0, ncb, x_tiles, nchunks); break;
        default: proj_fwd_bf16_kernel<MS, 3, LO><<<grid, 256, 0, st>>>(uh, ul, bst, phi, Nk, Nx, Nb, cols, col0, ncb, x_tiles, nchunks); break;
    }
    return hipGetLastError();
}

template <int MS, bool LO>
hipError_t fwd_bf16_res_nt(int NT, dim3 grid, size_t lds, hipStream_t st, const u16* uh, const u16* ul,
                           const unsigned char* bst, void* phi, int Nk, int Nx, int Nb, int cols, int col0, int ncb,
                           int x_tiles, int nchunks, int groups, int tiles) {
#define OCEAN_FWDB_RES(nt) \
    proj_fwd_bf16_res_kernel<MS, nt, LO><<<grid, 256, lds, st>>>(uh, ul, bst, phi, Nk, Nx, Nb, cols, col0, ncb, \
                                                                  x_tiles, nchunks, groups, tiles)
    switch (NT) {
        case 1: OCEAN_FWDB_RES(1); break;
        case 2: OCEAN_FWDB_RES(2); break;
        default: OCEAN_FWDB_RES(3); break;
    }
#undef OCEAN_FWDB_RES
    return hipGetLastError();
}

template <int W, bool LO>
hipError_t bwd_bf16_w(int NT, dim3 grid, hipStream_t st, const u16* uh, const u16* ul, const void* phi,
                      double* part, int Nk, int Nx, int NxP, int Nb, int cols, int col0, int ncb, int bb, int S,
                      int chunk) {
    switch (NT) {
        case 1: proj_bwd_bf16_kernel<1, W, LO><<<grid, 64 * W, 0, st>>>(uh, ul, phi, part, Nk, Nx, NxP, Nb, cols, col0, ncb, bb, S, chunk); break;
        case 2: proj_bwd_bf16_kernel<2, W, LO><<<grid, 64 * W, 0, st>>>(uh, ul, phi, part, Nk, Nx, NxP, Nb, cols, col0, ncb, bb, S, chunk); break;
        default: proj_bwd_bf16_kernel<3, W, LO><<<grid, 64 * W, 0, st>>>(uh, ul, phi, part, Nk, Nx, NxP, Nb, cols, col0, ncb, bb, S, chunk); break;
    }
    return hipGetLastError();
}

template <bool LO>
hipError_t bwd_bf16(int W, int NT, dim3 grid, hipStream_t st, const u16* uh, const u16* ul, const void* phi,
                    double* part, int Nk, int Nx, int NxP, int Nb, int cols, int col0, int ncb, int bb, int S,
                    int chunk) {
    switch (W) {
#define OCEAN_BWD_BF(w) \
        case w: return bwd_bf16_w<w, LO>(NT, grid, st, uh, ul, phi, part, Nk, Nx, NxP, Nb, cols, col0, ncb, bb, S, chunk);
        OCEAN_BWD_BF(1) OCEAN_BWD_BF(2) OCEAN_BWD_BF(3) OCEAN_BWD_BF(4) OCEAN_BWD_BF(5) OCEAN_BWD_BF(6)
        OCEAN_BWD_BF(7)
#undef OCEAN_BWD_BF
        default: return bwd_bf16_w<8, LO>(NT, grid, st, uh, ul, phi, part, Nk, Nx, NxP, Nb, cols, col0, ncb, bb, S, chunk);
    }
}

}  // namespace

hipError_t launch_proj_fwd_bf16(ocean_bse_s* h, const double* x, int nv, int col0, int ncb) {
    // 16 * MS rows per wave, 64 * MS per block
    const int MS = h->fwd_ms == 1 ? 1 : h->fwd_ms == 4 ? 4 : 2;
    const int cols = nv * h->Nc;
    const int NT = (2 * ncb + 15) / 16;
    const int x_tiles = (h->Nx + 64 * MS - 1) / (64 * MS);
    dim3 grid((unsigned)(h->Nk * x_tiles));
    hipError_t e;
    // stage the B operand of this pass once for all (k, band chunk)
    const int KC = fwd_band_chunk(h);
    const int nchunks = (h->Nb + KC - 1) / KC;
    int slot = prof_begin(h, "prep_b");
    const long long items = (long long)h->Nk * nchunks * (KC / 16) * NT * 64;
    const unsigned nblk = (unsigned)std::min<long long>((items + 255) / 256, 16384);
    prep_fwd_b_bf16_kernel<<<nblk, 256, 0, h->stream>>>(reinterpret_cast<const double2*>(x), h->ws.bst, h->Nk,
                                                        h->Nb, h->Nc, col0, ncb, NT, nchunks);
    e = hipGetLastError();
    prof_end(h, slot);
    if (e != hipSuccess) return e;
    slot = prof_begin(h, "proj_fwd");
    const u16* uh = reinterpret_cast<const u16*>(h->Ubf);
    const u16* ul = uh + (size_t)2 * h->Nk * h->Nx * h->Nb;
    const unsigned char* bst = h->ws.bst;
    const bool lo = h->precision == OCEAN_PREC_SPLIT_BF16;
    // phi offsets from a block's first row are 32-bit: a block's rows must span less than
    // 2 GiB of phi (x-blocks of 16 points, each Nk kXB cols elements apart)
    const size_t xb_bytes = (size_t)h->Nk * kXB * cols * (lo ? 8 : 4);
    const size_t row_tile_bytes = (size_t)(64 * MS / kXB) * xb_bytes;
    if (row_tile_bytes >= (1ull << 31)) {
        prof_end(h, slot);
        return hipErrorInvalidValue;
    }
    const size_t res_lds = h->fwd_tiles > 0 ? fwd_res_lds_bytes(h, ncb) : 0;
    if (res_lds > 0) {
        // the resident-B form: `tiles` x tiles per block
        const int tiles = std::max(1, std::min({h->fwd_tiles, x_tiles, (int)((1ull << 31) / row_tile_bytes)}));
        const int groups = (x_tiles + tiles - 1) / tiles;
        dim3 rgrid((unsigned)((long long)h->Nk * groups));
#define OCEAN_FWDB_RES_ARGS NT, rgrid, res_lds, h->stream, uh, ul, bst, h->ws.phi, h->Nk, h->Nx, h->Nb, cols, col0, ncb, \
                            x_tiles, nchunks, groups, tiles
        if (MS == 1)
            e = lo ? fwd_bf16_res_nt<1, true>(OCEAN_FWDB_RES_ARGS) : fwd_bf16_res_nt<1, false>(OCEAN_FWDB_RES_ARGS);
        else if (MS == 2)
            e = lo ? fwd_bf16_res_nt<2, true>(OCEAN_FWDB_RES_ARGS) : fwd_bf16_res_nt<2, false>(OCEAN_FWDB_RES_ARGS);
        else
            e = lo ? fwd_bf16_res_nt<4, true>(OCEAN_FWDB_RES_ARGS) : fwd_bf16_res_nt<4, false>(OCEAN_FWDB_RES_ARGS);
#undef OCEAN_FWDB_RES_ARGS
        prof_end(h, slot);
        return e;
    }
    if (MS == 1)
        e = lo ? fwd_bf16_nt<1, true>(NT, grid, h->stream, uh, ul, bst, h->ws.phi, h->Nk, h->Nx, h->Nb, cols, col0, ncb, x_tiles, nchunks)
               : fwd_bf16_nt<1, false>(NT, grid, h->stream, uh, ul, bst, h->ws.phi, h->Nk, h->Nx, h->Nb, cols, col0, ncb, x_tiles, nchunks);
    else if (MS == 2)
        e = lo ? fwd_bf16_nt<2, true>(NT, grid, h->stream, uh, ul, bst, h->ws.phi, h->Nk, h->Nx, h->Nb, cols, col0, ncb, x_tiles, nchunks)
               : fwd_bf16_nt<2, false>(NT, grid, h->stream, uh, ul, bst, h->ws.phi, h->Nk, h->Nx, h->Nb, cols, col0, ncb, x_tiles, nchunks);
    else
        e = lo ? fwd_bf16_nt<4, true>(NT, grid, h->stream, uh, ul, bst, h->ws.phi, h->Nk, h->Nx, h->Nb, cols, col0, ncb, x_tiles, nchunks)
               : fwd_bf16_nt<4, false>(NT, grid, h->stream, uh, ul, bst, h->ws.phi, h->Nk, h->Nx, h->Nb, cols, col0, ncb, x_tiles, nchunks);
    prof_end(h, slot);
    return e;
}

hipError_t launch_proj_bwd_bf16(ocean_bse_s* h, int nv, int col0, int ncb) {
    const int cols = nv * h->Nc;
    const int NT = (2 * ncb + 15) / 16;
    int bb, S, chunk;
    bwd_geometry(h, &bb, &S, &chunk);
    const int W = bwd_waves(h);
    dim3 grid((unsigned)(((long long)h->Nk * bb * S + 7) / 8 * 8));   // 8 XCDs, whole rounds
    const int slot = prof_begin(h, "proj_bwd");
    hipError_t e;
    const u16* uh = reinterpret_cast<const u16*>(h->UbfT);
    const u16* ul = uh + (size_t)2 * h->Nk * h->Nb * h->NxP;
    e = h->precision == OCEAN_PREC_SPLIT_BF16
            ? bwd_bf16<true>(W, NT, grid, h->stream, uh, ul, h->ws.phi, h->ws.part, h->Nk, h->Nx, h->NxP, h->Nb, cols, col0, ncb, bb, S, chunk)
            : bwd_bf16<false>(W, NT, grid, h->stream, uh, ul, h->ws.phi, h->ws.part, h->Nk, h->Nx, h->NxP, h->Nb, cols, col0, ncb, bb, S, chunk);
    prof_end(h, slot);
    return e;
}

hipError_t launch_u_to_bf16(ocean_bse_s* h, const double* src, long long g0, long long rows) {
    const bool split = h->precision == OCEAN_PREC_SPLIT_BF16;
    __bf16* hi = reinterpret_cast<__bf16*>(h->Ubf);
    __bf16* hiT = reinterpret_cast<__bf16*>(h->UbfT);
    __bf16* lo = split ? hi + (size_t)2 * h->Nk * h->Nx * h->Nb : nullptr;
    __bf16* loT = split ? hiT + (size_t)2 * h->Nk * h->Nb * h->NxP : nullptr;
    u_to_bf16_kernel<<<4096, 256, 0, h->stream>>>(src, g0, rows, h->Nx, h->Nb, h->NxP, phase_args(h), hi, lo, hiT, loT);
    return hipGetLastError();
}

}  // namespace ocean
