// Band projections of Algorithm 1 (section 3.2.1) on the gfx950 matrix cores, FP64 and FP32
// (the bf16 forms are in proj_bf16.hip).
//
//   band -> real space:  phi[k][x][col]      = sum_n u~[k][x][n] psi[k][n][col]
//   real space -> band:  part[s][k][n][col]  = sum_{x in chunk s} conj(u~[k][x][n]) phi'[k][x][col]
//
// u~ = e^{ik.x} u is the stored copy (a borrowed FP64 u is used as given and the k-grid
// transform applies the phase).  Both contractions are written as real GEMMs on the
// interleaved (re, im) storage: the contraction index is (band or point, re/im part) and
// the real output columns are (column, re/im), so the MFMA tiles consume the data in place:
//
//   forward  C[(x)][(c,q)] = sum_{(n,p)} U_p[x][n] B[(n,p)][(c,q)]
//            B = [[re psi, im psi], [-im psi, re psi]]        (rows p = 0, 1; columns q = 0, 1)
//   backward Z[(n)][(c,q)] = sum_{(x,p)} U_p[x][n] B[(x,p)][(c,q)]
//            B = [[re phi, im phi], [im phi, -re phi]]
//
// 16x16x4 MFMA: lane l = i + 16 kq holds A[i][kq] and B[kq][i]; result register r holds
// column i of row 4 r + kq (f64) or 4 kq + r (f32), as measured on gfx950.  A sub-step covers
// 8 contraction points: lane group kq holds points 2 kq and 2 kq + 1, and MFMA s = 0..3 of the
// sub-step contracts (point 2 kq + s / 2, part s % 2).
#include "internal.h"

namespace ocean {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> struct Cplx;
template <> struct Cplx<double> { typedef double2 c2; typedef v4d acc; };
template <> struct Cplx<float> { typedef float2 c2; typedef v4f acc; };

// Row of the 16x16 result held in accumulator register r of a lane in group kq
// (column = lane % 16).  The f64 and f32 16x16x4 instructions differ here.
template <typename T> __device__ __forceinline__ int acc_row(int kq, int r);
template <> __device__ __forceinline__ int acc_row<double>(int kq, int r) { return 4 * r + kq; }
template <> __device__ __forceinline__ int acc_row<float>(int kq, int r) { return 4 * kq + r; }

// B operands are staged in LDS in MFMA order: value s (0..3) of lane l for sub-step ss and
// column tile t sits at ((ss * NT + t) * 64 + l) * 4 + s, so a wave reads its operands with
// one 4-wide LDS load per (ss, t).  Lane l = i + 16 kq of sub-step ss covers the
// contraction slots (2 kq + s / 2, s % 2) of that 8-wide step and real column 16 t + i.

template <typename T> struct Vec4;
template <> struct Vec4<double> { typedef double4 t; };
template <> struct Vec4<float> { typedef float4 t; };

// Write the four B values of one complex input (re, im) at contraction point r8 (0..7 within
// a sub-step) and local column cl into the MFMA-ordered buffer.  fwd = true gives
// [[re, im], [-im, re]], false gives [[re, im], [im, -re]] (rows p, columns q).
template <typename T, int NT>
__device__ __forceinline__ void stage_pair(T* buf, int ss, int r8, int cl, double re, double im, bool fwd) {
    const int kq = r8 >> 1, ns = r8 & 1;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int jr = 2 * cl + q;
        const int t = jr >> 4, i = jr & 15;
        if (t >= NT) continue;
        T* dst = buf + ((size_t)(ss * NT + t) * 64 + i + 16 * kq) * 4 + 2 * ns;
        if (fwd) {
            dst[0] = (T)(q ? im : re);
            dst[1] = (T)(q ? re : -im);
        } else {
            dst[0] = (T)(q ? im : re);
            dst[1] = (T)(q ? -re : im);
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Forward projection.  Block = 4 waves and one k; wave w owns rows
// [xt*64*MS + w*16*MS, +16*MS) and every column tile.  The bands are walked in chunks of
// KC: the psi chunk (B operand, shared by all waves) is staged in LDS in MFMA order, double
// buffered, while each wave keeps the u values (A operand) of the next chunk in flight.
template <typename T, int MS, int NT, int KC>
__global__ __launch_bounds__(256) void proj_fwd_kernel(
    const typename Cplx<T>::c2* __restrict__ U, const double2* __restrict__ psi,
    typename Cplx<T>::c2* __restrict__ phi, int Nk, int Nx, int Nb, int Nc, int cols, int col0,
    int ncb, int x_tiles) {
    typedef typename Cplx<T>::c2 C2;
    typedef typename Cplx<T>::acc ACC;
    typedef typename Vec4<T>::t V4;
    constexpr int SS = KC / 8;                 // 8-band sub-steps per chunk
    constexpr int BUF = SS * NT * 64 * 4;      // T values per staged chunk
    __shared__ __align__(16) T sB[2][BUF];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const int k = blockIdx.x / x_tiles;
    const int xt = blockIdx.x - k * x_tiles;
    const int rowbase = xt * (64 * MS) + wave * (16 * MS);
    const C2* Uk = U + (size_t)k * Nx * Nb;

    // u rows of this block: [xt*64*MS, min(Nx, (xt+1)*64*MS)), all bands
    const int brow0 = xt * (64 * MS);
    const int brows = min(Nx - brow0, 64 * MS);
    const Rsrc ur = make_rsrc(Uk + (size_t)brow0 * Nb, (size_t)brows * Nb * sizeof(C2));
    const Rsrc pr = make_rsrc(psi, (size_t)(col0 + ncb + Nc) / Nc * Nk * Nb * Nc * sizeof(double2));
    bool rval[MS];
    unsigned urow[MS];
#pragma unroll
    for (int ms = 0; ms < MS; ++ms) {
        const int row = rowbase + 16 * ms + i;
        rval[ms] = row < Nx;
        urow[ms] = (unsigned)((row - brow0) * Nb) * sizeof(C2);
    }
    // cooperative psi chunk loads: element e = (n_local, c_local), c fastest
    constexpr int PER = (KC * kColsPerPass + 255) / 256;
    auto load_p = [&](int n0, double2 (&pv)[PER]) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = threadIdx.x + 256 * j;
            const int nl = e / kColsPerPass, cl = e - nl * kColsPerPass;
            const int n = n0 + nl;
            const bool ok = nl < KC && cl < ncb && n < Nb;
            const int col = col0 + cl;
            const int vv = col / Nc, c = col - vv * Nc;
            const unsigned off = (unsigned)((((size_t)(vv * Nk + k) * Nb + n) * Nc + c) * sizeof(double2));
            pv[j] = bload<double2>(pr, ok ? off : kOob);
        }
    };
    auto store_p = [&](int buf, const double2 (&pv)[PER]) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = threadIdx.x + 256 * j;
            const int nl = e / kColsPerPass, cl = e - nl * kColsPerPass;
            if (nl < KC && cl < ncb) stage_pair<T, NT>(sB[buf], nl >> 3, nl & 7, cl, pv[j].x, pv[j].y, true);
        }
    };
    auto load_a = [&](int n0, C2 (&aa)[MS][SS][2]) {
#pragma unroll
        for (int ss = 0; ss < SS; ++ss)
#pragma unroll
            for (int ns = 0; ns < 2; ++ns) {
                const int n = n0 + 8 * ss + 2 * kq + ns;
                const bool nok = n < Nb;
#pragma unroll
                for (int ms = 0; ms < MS; ++ms)
                    aa[ms][ss][ns] = bload<C2>(ur, (nok && rval[ms]) ? urow[ms] + (unsigned)(n * sizeof(C2)) : kOob);
            }
    };

    // padding columns stay zero in both buffers
    for (int e = threadIdx.x; e < 2 * BUF; e += 256) (&sB[0][0])[e] = (T)0;

    ACC acc[MS][NT];
#pragma unroll
    for (int ms = 0; ms < MS; ++ms)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[ms][t] = ACC{0, 0, 0, 0};

    C2 a[MS][SS][2], an[MS][SS][2];
    double2 pv[PER];
    load_p(0, pv);
    load_a(0, a);
    // Drain the prologue loads here: otherwise the wait-count analysis merges this path into
    // the loop header and waits for every in-flight prefetch before the first MFMA of a chunk.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    store_p(0, pv);
    int buf = 0;
    for (int n0 = 0; n0 < Nb; n0 += KC) {
        __syncthreads();
        // next chunk (masked to zero past the last band); the scheduling barrier keeps these
        // loads at the top so that they overlap the MFMAs of the current chunk
        load_p(n0 + KC, pv);
        load_a(n0 + KC, an);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ss = 0; ss < SS; ++ss) {
            V4 bv[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t)
                bv[t] = *reinterpret_cast<const V4*>(&sB[buf][((ss * NT + t) * 64 + lane) * 4]);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
#pragma unroll
                for (int ms = 0; ms < MS; ++ms) {
                    const T av = (s & 1) ? a[ms][ss][s >> 1].y : a[ms][ss][s >> 1].x;
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const T b = s == 0 ? bv[t].x : s == 1 ? bv[t].y : s == 2 ? bv[t].z : bv[t].w;
                        acc[ms][t] = mfma16(av, b, acc[ms][t]);
                    }
                }
            }
        }
        store_p(buf ^ 1, pv);
#pragma unroll
        for (int ms = 0; ms < MS; ++ms)
#pragma unroll
            for (int ss = 0; ss < SS; ++ss) {
                a[ms][ss][0] = an[ms][ss][0];
                a[ms][ss][1] = an[ms][ss][1];
            }
        buf ^= 1;
    }

    T* out = reinterpret_cast<T*>(phi);
#pragma unroll
    for (int ms = 0; ms < MS; ++ms)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int jr = 16 * t + i;
            if ((jr >> 1) >= ncb) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rowbase + 16 * ms + acc_row<T>(kq, r);
                if (row < Nx)
                    out[2 * phi_index_x(row, col0, k, Nk, cols) + jr] = acc[ms][t][r];
            }
        }
}

// ---------------------------------------------------------------------------------------------
// Backward projection with split-K over x.  Block = (k, band block of W x 16 bands,
// x chunk); wave w owns the 16 bands [band block * 16 W + 16 w, +16).  The chunk is walked
// in tiles of XT points: the phi' tile (B operand, shared by all waves) is staged in LDS in
// MFMA order, double buffered, and every wave keeps the u values of the next tile in flight.
template <typename T, int NT, int XT, int W>
__global__ __launch_bounds__(64 * W) void proj_bwd_kernel(
    const typename Cplx<T>::c2* __restrict__ U, const typename Cplx<T>::c2* __restrict__ phi,
    double* __restrict__ part, int Nk, int Nx, int Nb, int cols, int col0, int ncb,
    int band_blocks, int S, int chunk) {
    typedef typename Cplx<T>::c2 C2;
    typedef typename Cplx<T>::acc ACC;
    typedef typename Vec4<T>::t V4;
    constexpr int SS = XT / 8;
    constexpr int BUF = SS * NT * 64 * 4;
    __shared__ __align__(16) T sB[2][BUF];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    int blk = blockIdx.x;
    const int s = blk % S;
    blk /= S;
    const int bb = blk % band_blocks;
    const int k = blk / band_blocks;
    const int nbase = bb * 16 * W + 16 * wave;
    const int x_begin = s * chunk;
    const int x_end = min(Nx, x_begin + chunk);
    const C2* Uk = U + (size_t)k * Nx * Nb;

    const int n = nbase + i;
    const bool nval = n < Nb;
    // u rows [x_begin, x_end) of this k, all bands; phi' x-blocks covering the chunk
    const Rsrc ur = make_rsrc(Uk + (size_t)x_begin * Nb, (size_t)(x_end - x_begin) * Nb * sizeof(C2));
    const int xb0 = x_begin / kXB;
    const C2* pbase = phi + (size_t)xb0 * Nk * kXB * cols;
    const Rsrc prs = make_rsrc(pbase, (size_t)((x_end - 1) / kXB - xb0 + 1) * Nk * kXB * cols * sizeof(C2));

    constexpr int PER = (XT * kColsPerPass + 64 * W - 1) / (64 * W);
    auto load_b = [&](int x0, C2 (&bv)[PER]) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = threadIdx.x + 64 * W * j;
            const int xl = e / kColsPerPass, cl = e - xl * kColsPerPass;
            const int x = x0 + xl;
            const bool ok = xl < XT && cl < ncb && x < x_end;
            const unsigned off = (unsigned)((phi_index_x(x, col0 + cl, k, Nk, cols) - (size_t)xb0 * Nk * kXB * cols) * sizeof(C2));
            bv[j] = bload<C2>(prs, ok ? off : kOob);
        }
    };
    auto store_b = [&](int buf, const C2 (&bv)[PER]) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = threadIdx.x + 64 * W * j;
            const int xl = e / kColsPerPass, cl = e - xl * kColsPerPass;
            if (xl < XT && cl < ncb) stage_pair<T, NT>(sB[buf], xl >> 3, xl & 7, cl, bv[j].x, bv[j].y, false);
        }
    };
    auto load_a = [&](int x0, C2 (&aa)[SS][2]) {
#pragma unroll
        for (int ss = 0; ss < SS; ++ss)
#pragma unroll
            for (int xs = 0; xs < 2; ++xs) {
                const int x = x0 + 8 * ss + 2 * kq + xs;
                const bool ok = nval && x < x_end;
                aa[ss][xs] = bload<C2>(ur, ok ? (unsigned)(((x - x_begin) * Nb + n) * sizeof(C2)) : kOob);
            }
    };

    for (int e = threadIdx.x; e < 2 * BUF; e += 64 * W) (&sB[0][0])[e] = (T)0;

    ACC acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = ACC{0, 0, 0, 0};

    C2 a[SS][2], an[SS][2];
    C2 bl[PER];
    load_b(x_begin, bl);
    load_a(x_begin, a);
    __builtin_amdgcn_s_waitcnt(0);  // drain the prologue (see the forward kernel)
    __syncthreads();
    store_b(0, bl);
    int buf = 0;
    for (int x0 = x_begin; x0 < x_end; x0 += XT) {
        __syncthreads();
        // next tile (masked to zero past the chunk end), kept ahead of the MFMAs
        load_b(x0 + XT, bl);
        load_a(x0 + XT, an);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ss = 0; ss < SS; ++ss) {
            V4 bv[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t)
                bv[t] = *reinterpret_cast<const V4*>(&sB[buf][((ss * NT + t) * 64 + lane) * 4]);
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const T av = (st & 1) ? a[ss][st >> 1].y : a[ss][st >> 1].x;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const T b = st == 0 ? bv[t].x : st == 1 ? bv[t].y : st == 2 ? bv[t].z : bv[t].w;
                    acc[t] = mfma16(av, b, acc[t]);
                }
            }
        }
        store_b(buf ^ 1, bl);
#pragma unroll
        for (int ss = 0; ss < SS; ++ss) {
            a[ss][0] = an[ss][0];
            a[ss][1] = an[ss][1];
        }
        buf ^= 1;
    }

    double* out = part + ((size_t)s * Nk + k) * Nb * 2 * cols + 2 * col0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int jr = 16 * t + i;
        if ((jr >> 1) >= ncb) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int nn = nbase + acc_row<T>(kq, r);
            if (nn < Nb) out[(size_t)nn * 2 * cols + jr] = (double)acc[t][r];
        }
    }
}

template <typename T> struct Tiles;
template <> struct Tiles<double> { static constexpr int KC = 16, XT = 32; };
template <> struct Tiles<float> { static constexpr int KC = 32, XT = 64; };

template <typename T, int MS>
hipError_t fwd_dispatch_nt(int NT, dim3 grid, hipStream_t st, const void* U, const double* x,
                           void* phi, int Nk, int Nx, int Nb, int Nc, int cols, int col0, int ncb,
                           int x_tiles) {
    typedef typename Cplx<T>::c2 C2;
    const C2* u = static_cast<const C2*>(U);
    C2* p = static_cast<C2*>(phi);
    const double2* ps = reinterpret_cast<const double2*>(x);
    switch (NT) {
        case 1: proj_fwd_kernel<T, MS, 1, Tiles<T>::KC><<<grid, 256, 0, st>>>(u, ps, p, Nk, Nx, Nb, Nc, cols, col0, ncb, x_tiles); break;
        case 2: proj_fwd_kernel<T, MS, 2, Tiles<T>::KC><<<grid, 256, 0, st>>>(u, ps, p, Nk, Nx, Nb, Nc, cols, col0, ncb, x_tiles); break;
        default: proj_fwd_kernel<T, MS, 3, Tiles<T>::KC><<<grid, 256, 0, st>>>(u, ps, p, Nk, Nx, Nb, Nc, cols, col0, ncb, x_tiles); break;
    }
    return hipGetLastError();
}

template <typename T, int W>
hipError_t bwd_dispatch_w(int NT, dim3 grid, hipStream_t st, const void* U, const void* phi,
                          double* part, int Nk, int Nx, int Nb, int cols, int col0, int ncb, int bb,
                          int S, int chunk) {
    typedef typename Cplx<T>::c2 C2;
    constexpr int XT = Tiles<T>::XT;
    const C2* u = static_cast<const C2*>(U);
    const C2* p = static_cast<const C2*>(phi);
    switch (NT) {
        case 1: proj_bwd_kernel<T, 1, XT, W><<<grid, 64 * W, 0, st>>>(u, p, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk); break;
        case 2: proj_bwd_kernel<T, 2, XT, W><<<grid, 64 * W, 0, st>>>(u, p, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk); break;
        default: proj_bwd_kernel<T, 3, XT, W><<<grid, 64 * W, 0, st>>>(u, p, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t bwd_dispatch(int W, int NT, dim3 grid, hipStream_t st, const void* U, const void* phi,
                        double* part, int Nk, int Nx, int Nb, int cols, int col0, int ncb, int bb,
                        int S, int chunk) {
    switch (W) {
#define OCEAN_BWD_W(w) \
        case w: return bwd_dispatch_w<T, w>(NT, grid, st, U, phi, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk);
        OCEAN_BWD_W(1) OCEAN_BWD_W(2) OCEAN_BWD_W(3) OCEAN_BWD_W(4) OCEAN_BWD_W(5) OCEAN_BWD_W(6)
        OCEAN_BWD_W(7)
#undef OCEAN_BWD_W
        default: return bwd_dispatch_w<T, 8>(NT, grid, st, U, phi, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk);
    }
}

}  // namespace


// Backward-projection geometry: band blocks of up to 8 waves x 16 bands, and x chunks
// (multiples of 8 points) so that the grid holds about bwd_target_blocks blocks.
int bwd_waves(int Nb) {
    const int nb16 = (Nb + 15) / 16;
    return nb16 < 8 ? nb16 : 8;
}

void bwd_geometry_for(const ocean_bse_s* h, int target_blocks, int* band_blocks, int* S, int* chunk) {
    const int W = bwd_waves(h->Nb);
    const int bb = (h->Nb + 16 * W - 1) / (16 * W);
    const long long per_chunk = (long long)h->Nk * bb;
    long long s = (target_blocks + per_chunk - 1) / per_chunk;
    const long long smax = std::max(1, (h->Nx + 511) / 512);  // >= 512 points per chunk
    if (s < 1) s = 1;
    if (s > smax) s = smax;
    int c = (int)((h->Nx + s - 1) / s);
    c = (c + 7) / 8 * 8;
    *chunk = c;
    *S = (h->Nx + c - 1) / c;
    *band_blocks = bb;
}

void bwd_geometry(const ocean_bse_s* h, int* band_blocks, int* S, int* chunk) {
    bwd_geometry_for(h, h->bwd_target_blocks, band_blocks, S, chunk);
}

bool is_bf16_mode(int precision) {
    return precision == OCEAN_PREC_SPLIT_BF16 || precision == OCEAN_PREC_BF16;
}

int fwd_band_chunk(const ocean_bse_s* h) { return is_bf16_mode(h->precision) ? 32 : 0; }

hipError_t launch_proj_fwd(ocean_bse_s* h, const double* x, int nv, int col0, int ncb) {
    if (is_bf16_mode(h->precision)) return launch_proj_fwd_bf16(h, x, nv, col0, ncb);
    const int MS = h->fwd_ms == 1 ? 1 : 2;   // 16 * MS rows per wave, 64 * MS per block
    const int cols = nv * h->Nc;
    const int NT = (2 * ncb + 15) / 16;
    const int x_tiles = (h->Nx + 64 * MS - 1) / (64 * MS);
    dim3 grid((unsigned)(h->Nk * x_tiles));
    hipError_t e;
    const int slot = prof_begin(h, "proj_fwd");
    if (h->precision == OCEAN_PREC_FP64)
        e = MS == 1 ? fwd_dispatch_nt<double, 1>(NT, grid, h->stream, h->U64, x, h->ws.phi, h->Nk, h->Nx,
                                                 h->Nb, h->Nc, cols, col0, ncb, x_tiles)
                    : fwd_dispatch_nt<double, 2>(NT, grid, h->stream, h->U64, x, h->ws.phi, h->Nk, h->Nx,
                                                 h->Nb, h->Nc, cols, col0, ncb, x_tiles);
    else
        e = MS == 1 ? fwd_dispatch_nt<float, 1>(NT, grid, h->stream, h->U32, x, h->ws.phi, h->Nk, h->Nx,
                                                h->Nb, h->Nc, cols, col0, ncb, x_tiles)
                    : fwd_dispatch_nt<float, 2>(NT, grid, h->stream, h->U32, x, h->ws.phi, h->Nk, h->Nx,
                                                h->Nb, h->Nc, cols, col0, ncb, x_tiles);
    prof_end(h, slot);
    return e;
}

hipError_t launch_proj_bwd(ocean_bse_s* h, int nv, int col0, int ncb) {
    if (is_bf16_mode(h->precision)) return launch_proj_bwd_bf16(h, nv, col0, ncb);
    const int cols = nv * h->Nc;
    const int NT = (2 * ncb + 15) / 16;
    int bb, S, chunk;
    bwd_geometry(h, &bb, &S, &chunk);
    const int W = bwd_waves(h->Nb);
    dim3 grid((unsigned)((long long)h->Nk * bb * S));
    const int slot = prof_begin(h, "proj_bwd");
    hipError_t e;
    if (h->precision == OCEAN_PREC_FP64)
        e = bwd_dispatch<double>(W, NT, grid, h->stream, h->U64, h->ws.phi, h->ws.part, h->Nk,
                                 h->Nx, h->Nb, cols, col0, ncb, bb, S, chunk);
    else
        e = bwd_dispatch<float>(W, NT, grid, h->stream, h->U32, h->ws.phi, h->ws.part, h->Nk,
                                h->Nx, h->Nb, cols, col0, ncb, bb, S, chunk);
    prof_end(h, slot);
    return e;
}

}  // namespace ocean
