// Band projections of Algorithm 1 (section 3.2.1) on the gfx950 matrix cores.
//
//   forward (line 2):  phi[k][x][col]  = sum_n u[k][x][n] psi[k][n][col]
//   backward (line 6): part[s][k][n][col] = sum_{x in chunk s} conj(u[k][x][n]) phi'[k][x][col]
//
// The e^{+-ik.x} phases of lines 2 and 6 are applied by the k-grid transform
// kernel, so u is used exactly as stored.  Both contractions are written as
// real GEMMs on the interleaved (re, im) storage of u: the contraction index is
// (band or point, re/im part) and the real output columns are (column, re/im),
// so one 16x16x4 MFMA tile consumes the complex data in place:
//
//   forward  C[(x)][(c,q)] = sum_{(n,p)} U_p[x][n] B[(n,p)][(c,q)]
//            B = [[re psi, im psi], [-im psi, re psi]]        (rows p = 0, 1; columns q = 0, 1)
//   backward Z[(n)][(c,q)] = sum_{(x,p)} U_p[x][n] B[(x,p)][(c,q)]
//            B = [[re phi, im phi], [im phi, -re phi]]
//
// MFMA operand layout (v_mfma_{f64,f32}_16x16x4): lane l = i + 16 kq holds
// A[i][kq] and B[kq][i]; result register r of lane l holds column i of row
// 4 r + kq (f64) or 4 kq + r (f32), as measured on gfx950.  Inside one 16x16x4 step the four K slots kq map to the contraction
// index ((2 kq + s/2), s%2) for step s = 0..3, so every lane reads two adjacent
// complex values of u (32 contiguous bytes in FP64).
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

template <typename C2> __device__ __forceinline__ C2 czero() { C2 z; z.x = 0; z.y = 0; return z; }

// Row of the 16x16 result held in accumulator register r of a lane in group kq
// (column = lane % 16).  The f64 and f32 16x16x4 instructions differ here.
template <typename T> __device__ __forceinline__ int acc_row(int kq, int r);
template <> __device__ __forceinline__ int acc_row<double>(int kq, int r) { return 4 * r + kq; }
template <> __device__ __forceinline__ int acc_row<float>(int kq, int r) { return 4 * kq + r; }

// ---------------------------------------------------------------------------------------------
// Forward projection.  Block = 4 waves; wave w owns rows [xt*64*MS + w*16*MS, +16*MS) of one k.
template <typename T, int MS, int NT>
__global__ __launch_bounds__(256) void proj_fwd_kernel(
    const typename Cplx<T>::c2* __restrict__ U, const double2* __restrict__ psi,
    typename Cplx<T>::c2* __restrict__ phi, int Nk, int Nx, int Nb, int Nc, int cols, int col0,
    int ncb, int x_tiles) {
    typedef typename Cplx<T>::c2 C2;
    typedef typename Cplx<T>::acc ACC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const int k = blockIdx.x / x_tiles;
    const int xt = blockIdx.x - k * x_tiles;
    const int rowbase = xt * (64 * MS) + wave * (16 * MS);
    const C2* Uk = U + (size_t)k * Nx * Nb;
    const int q = i & 1;

    const double2* pcol[NT];
    bool cval[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int cl = (16 * t + i) >> 1;
        cval[t] = cl < ncb;
        const int col = col0 + (cval[t] ? cl : 0);
        const int v = col / Nc, c = col - v * Nc;
        pcol[t] = psi + ((size_t)(v * Nk + k) * Nb) * Nc + c;
    }
    bool rval[MS];
    const C2* urow[MS];
#pragma unroll
    for (int ms = 0; ms < MS; ++ms) {
        const int row = rowbase + 16 * ms + i;
        rval[ms] = row < Nx;
        urow[ms] = Uk + (size_t)(rval[ms] ? row : 0) * Nb;
    }

    ACC acc[MS][NT];
#pragma unroll
    for (int ms = 0; ms < MS; ++ms)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[ms][t] = ACC{0, 0, 0, 0};

    for (int n0 = 0; n0 < Nb; n0 += 8) {
        C2 a[MS][2];
        T bv[NT][4];
#pragma unroll
        for (int ns = 0; ns < 2; ++ns) {
            const int n = n0 + 2 * kq + ns;
            const bool nok = n < Nb;
#pragma unroll
            for (int ms = 0; ms < MS; ++ms) a[ms][ns] = (nok && rval[ms]) ? urow[ms][n] : czero<C2>();
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                double2 p = (nok && cval[t]) ? pcol[t][(size_t)n * Nc] : czero<double2>();
                // B[(n, 0)][(c, q)] and B[(n, 1)][(c, q)]
                bv[t][2 * ns + 0] = (T)(q ? p.y : p.x);
                bv[t][2 * ns + 1] = (T)(q ? p.x : -p.y);
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int ms = 0; ms < MS; ++ms) {
                const T av = (s & 1) ? a[ms][s >> 1].y : a[ms][s >> 1].x;
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[ms][t] = mfma16(av, bv[t][s], acc[ms][t]);
            }
        }
    }

    T* out = reinterpret_cast<T*>(phi) + (size_t)k * Nx * 2 * cols + 2 * col0;
#pragma unroll
    for (int ms = 0; ms < MS; ++ms)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int jr = 16 * t + i;
            if ((jr >> 1) >= ncb) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rowbase + 16 * ms + acc_row<T>(kq, r);
                if (row < Nx) out[(size_t)row * 2 * cols + jr] = acc[ms][t][r];
            }
        }
}

// ---------------------------------------------------------------------------------------------
// Backward projection with split-K over x.  Block = (k, band block, x chunk); the four waves
// take interleaved groups of 8 points of the chunk and are summed through LDS in wave order.
template <typename T, int MS, int NT>
__global__ __launch_bounds__(256) void proj_bwd_kernel(
    const typename Cplx<T>::c2* __restrict__ U, const typename Cplx<T>::c2* __restrict__ phi,
    double* __restrict__ part, int Nk, int Nx, int Nb, int cols, int col0, int ncb,
    int band_blocks, int S, int chunk) {
    typedef typename Cplx<T>::c2 C2;
    typedef typename Cplx<T>::acc ACC;
    __shared__ ACC red[3][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    int blk = blockIdx.x;
    const int s = blk % S;
    blk /= S;
    const int bb = blk % band_blocks;
    const int k = blk / band_blocks;
    const int nbase = bb * 16 * MS;
    const int x_begin = s * chunk;
    const int x_end = min(Nx, x_begin + chunk);
    const C2* Uk = U + (size_t)k * Nx * Nb;
    const C2* Pk = phi + (size_t)k * Nx * cols;
    const int q = i & 1;

    int pcol[NT];
    bool cval[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int cl = (16 * t + i) >> 1;
        cval[t] = cl < ncb;
        pcol[t] = col0 + (cval[t] ? cl : 0);
    }
    bool nval[MS];
    int ncol[MS];
#pragma unroll
    for (int ms = 0; ms < MS; ++ms) {
        const int n = nbase + 16 * ms + i;
        nval[ms] = n < Nb;
        ncol[ms] = nval[ms] ? n : 0;
    }

    ACC acc[MS][NT];
#pragma unroll
    for (int ms = 0; ms < MS; ++ms)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[ms][t] = ACC{0, 0, 0, 0};

    for (int xb = x_begin + 8 * wave; xb < x_end; xb += 32) {
        C2 a[MS][2];
        T bv[NT][4];
#pragma unroll
        for (int xs = 0; xs < 2; ++xs) {
            const int x = xb + 2 * kq + xs;
            const bool xok = x < x_end;
            const C2* ur = Uk + (size_t)(xok ? x : 0) * Nb;
#pragma unroll
            for (int ms = 0; ms < MS; ++ms) a[ms][xs] = (xok && nval[ms]) ? ur[ncol[ms]] : czero<C2>();
            const C2* pr = Pk + (size_t)(xok ? x : 0) * cols;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                C2 p = (xok && cval[t]) ? pr[pcol[t]] : czero<C2>();
                // B[(x, 0)][(c, q)] and B[(x, 1)][(c, q)]
                bv[t][2 * xs + 0] = q ? p.y : p.x;
                bv[t][2 * xs + 1] = q ? -p.x : p.y;
            }
        }
#pragma unroll
        for (int st = 0; st < 4; ++st) {
#pragma unroll
            for (int ms = 0; ms < MS; ++ms) {
                const T av = (st & 1) ? a[ms][st >> 1].y : a[ms][st >> 1].x;
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[ms][t] = mfma16(av, bv[t][st], acc[ms][t]);
            }
        }
    }

    // deterministic cross-wave sum: ((w0 + w1) + w2) + w3
#pragma unroll
    for (int ms = 0; ms < MS; ++ms)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (wave > 0) red[wave - 1][lane] = acc[ms][t];
            __syncthreads();
            if (wave == 0) {
                ACC v = acc[ms][t];
                v += red[0][lane];
                v += red[1][lane];
                v += red[2][lane];
                acc[ms][t] = v;
            }
            __syncthreads();
        }
    if (wave != 0) return;

    double* out = part + ((size_t)s * Nk + k) * Nb * 2 * cols + 2 * col0;
#pragma unroll
    for (int ms = 0; ms < MS; ++ms)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int jr = 16 * t + i;
            if ((jr >> 1) >= ncb) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = nbase + 16 * ms + acc_row<T>(kq, r);
                if (n < Nb) out[(size_t)n * 2 * cols + jr] = (double)acc[ms][t][r];
            }
        }
}

template <typename T, int MS>
hipError_t fwd_dispatch_nt(int NT, dim3 grid, hipStream_t st, const void* U, const double* x,
                           void* phi, int Nk, int Nx, int Nb, int Nc, int cols, int col0, int ncb,
                           int x_tiles) {
    typedef typename Cplx<T>::c2 C2;
    const C2* u = static_cast<const C2*>(U);
    C2* p = static_cast<C2*>(phi);
    const double2* ps = reinterpret_cast<const double2*>(x);
    switch (NT) {
        case 1: proj_fwd_kernel<T, MS, 1><<<grid, 256, 0, st>>>(u, ps, p, Nk, Nx, Nb, Nc, cols, col0, ncb, x_tiles); break;
        case 2: proj_fwd_kernel<T, MS, 2><<<grid, 256, 0, st>>>(u, ps, p, Nk, Nx, Nb, Nc, cols, col0, ncb, x_tiles); break;
        default: proj_fwd_kernel<T, MS, 3><<<grid, 256, 0, st>>>(u, ps, p, Nk, Nx, Nb, Nc, cols, col0, ncb, x_tiles); break;
    }
    return hipGetLastError();
}

template <typename T, int MS>
hipError_t bwd_dispatch_nt(int NT, dim3 grid, hipStream_t st, const void* U, const void* phi,
                           double* part, int Nk, int Nx, int Nb, int cols, int col0, int ncb,
                           int bb, int S, int chunk) {
    typedef typename Cplx<T>::c2 C2;
    const C2* u = static_cast<const C2*>(U);
    const C2* p = static_cast<const C2*>(phi);
    switch (NT) {
        case 1: proj_bwd_kernel<T, MS, 1><<<grid, 256, 0, st>>>(u, p, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk); break;
        case 2: proj_bwd_kernel<T, MS, 2><<<grid, 256, 0, st>>>(u, p, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk); break;
        default: proj_bwd_kernel<T, MS, 3><<<grid, 256, 0, st>>>(u, p, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t bwd_dispatch(int MS, int NT, dim3 grid, hipStream_t st, const void* U, const void* phi,
                        double* part, int Nk, int Nx, int Nb, int cols, int col0, int ncb, int bb,
                        int S, int chunk) {
    switch (MS) {
        case 1: return bwd_dispatch_nt<T, 1>(NT, grid, st, U, phi, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk);
        case 2: return bwd_dispatch_nt<T, 2>(NT, grid, st, U, phi, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk);
        case 4: return bwd_dispatch_nt<T, 4>(NT, grid, st, U, phi, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk);
        case 6: return bwd_dispatch_nt<T, 6>(NT, grid, st, U, phi, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk);
        default: return bwd_dispatch_nt<T, 8>(NT, grid, st, U, phi, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk);
    }
}

}  // namespace

// Band-subtile count per wave for the backward projection: the smallest supported
// MS covering all bands (one band block), capped at 8.
int bwd_ms(int Nb) {
    const int nb16 = (Nb + 15) / 16;
    if (nb16 <= 1) return 1;
    if (nb16 <= 2) return 2;
    if (nb16 <= 4) return 4;
    if (nb16 <= 6) return 6;
    return 8;
}

void bwd_geometry(const ocean_bse_s* h, int* band_blocks, int* S, int* chunk) {
    const int ms = bwd_ms(h->Nb);
    const int bb = (h->Nb + 16 * ms - 1) / (16 * ms);
    const long long per_chunk = (long long)h->Nk * bb;
    long long s = (h->bwd_target_blocks + per_chunk - 1) / per_chunk;
    const long long smax = (h->Nx + 31) / 32;
    if (s < 1) s = 1;
    if (s > smax) s = smax;
    int c = (int)((h->Nx + s - 1) / s);
    c = (c + 31) / 32 * 32;
    *chunk = c;
    *S = (h->Nx + c - 1) / c;
    *band_blocks = bb;
}

hipError_t launch_proj_fwd(ocean_bse_s* h, const double* x, int nv, int col0, int ncb) {
    constexpr int MS = 2;
    const int cols = nv * h->Nc;
    const int NT = (2 * ncb + 15) / 16;
    const int x_tiles = (h->Nx + 64 * MS - 1) / (64 * MS);
    dim3 grid((unsigned)(h->Nk * x_tiles));
    const int slot = prof_begin(h, "proj_fwd");
    hipError_t e;
    if (h->precision == OCEAN_PREC_FP64)
        e = fwd_dispatch_nt<double, MS>(NT, grid, h->stream, h->U64, x, h->ws.phi, h->Nk, h->Nx,
                                        h->Nb, h->Nc, cols, col0, ncb, x_tiles);
    else
        e = fwd_dispatch_nt<float, MS>(NT, grid, h->stream, h->U32, x, h->ws.phi, h->Nk, h->Nx,
                                       h->Nb, h->Nc, cols, col0, ncb, x_tiles);
    prof_end(h, slot);
    return e;
}

hipError_t launch_proj_bwd(ocean_bse_s* h, int nv, int col0, int ncb) {
    const int cols = nv * h->Nc;
    const int NT = (2 * ncb + 15) / 16;
    int bb, S, chunk;
    bwd_geometry(h, &bb, &S, &chunk);
    const int ms = bwd_ms(h->Nb);
    dim3 grid((unsigned)((long long)h->Nk * bb * S));
    const int slot = prof_begin(h, "proj_bwd");
    hipError_t e;
    if (h->precision == OCEAN_PREC_FP64)
        e = bwd_dispatch<double>(ms, NT, grid, h->stream, h->U64, h->ws.phi, h->ws.part, h->Nk,
                                 h->Nx, h->Nb, cols, col0, ncb, bb, S, chunk);
    else
        e = bwd_dispatch<float>(ms, NT, grid, h->stream, h->U32, h->ws.phi, h->ws.part, h->Nk,
                                h->Nx, h->Nb, cols, col0, ncb, bb, S, chunk);
    prof_end(h, slot);
    return e;
}

}  // namespace ocean
