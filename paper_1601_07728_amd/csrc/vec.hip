// Vector-sized kernels of the H*v and of the Haydock recursion:
//   - the short-range local-basis term (section 3.2.2): projection in, the small
//     interaction matrix, projection out
//   - the diagonal (H_e) and core-matrix (-H_h) terms, summed with the back-projection
//     partials of the long-range W0 term into y (section 3.2: the pieces are summed)
//   - Lanczos inner products, updates and norms (section 3.2, Haydock), FP64 with a
//     fixed reduction order
//   - the continued-fraction spectrum (section 2, eq. loss.fcn)
//   - set-up: the W(x, R) table, precision copies of u, dipole initial vectors
#include "internal.h"

namespace ocean {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// Fixed-order block sum of one double per thread (blockDim.x = 256).
__device__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ double2 block_sum2(double2 v, double* sh) {
    const double re = block_sum(v.x, sh);
    const double im = block_sum(v.y, sh);
    return make_double2(re, im);
}

// ---- local term --------------------------------------------------------------------------------
// part[blk][v][c*Nmu+mu] = sum_{kn in rows of blk} A[kn][mu] x[v][kn][c].  A block takes R
// consecutive (k, n) rows (R from the LDS budget: 128 for the d channel, about 40 for 64
// channels): the A rows and, per vector, the x rows go to LDS with coalesced loads.  With
// NP = Nc Nmu <= 256 pairs, thread (pair, g) sums the rows r = g, g + G, ... of its pair and
// the G partial sums are added in a fixed order; with more pairs a thread takes pairs
// t, t + 256, ... over all rows.
constexpr int kLocRowsMax = 128;
constexpr int kLocLdsElems = 3072;   // complex elements of A and x rows staged per block (48 KiB)

int local_rows(int Nc, int Nmu) {
    const int r = kLocLdsElems / (Nmu + Nc);
    return r < kLocRowsMax ? r : kLocRowsMax;
}

__global__ __launch_bounds__(256) void local_in_kernel(const double2* __restrict__ x,
                                                       const double2* __restrict__ A,
                                                       double2* __restrict__ part, int nv,
                                                       long long NkNb, int Nc, int Nmu, int R) {
    extern __shared__ double2 lds[];
    double2* sA = lds;                 // [R][Nmu]
    double2* sX = lds + R * Nmu;       // [R][Nc]
    __shared__ double2 red[256];
    const int NP = Nc * Nmu;
    const int G = NP <= 256 ? 256 / NP : 1;
    const int t = threadIdx.x;
    const long long r0 = (long long)blockIdx.x * R;
    const int rows = (int)min((long long)R, NkNb - r0);
    for (int e = t; e < R * Nmu; e += 256)
        sA[e] = e < rows * Nmu ? A[r0 * Nmu + e] : make_double2(0.0, 0.0);
    for (int v = 0; v < nv; ++v) {
        const double2* xv = x + ((size_t)v * NkNb + r0) * Nc;
        for (int e = t; e < R * Nc; e += 256) sX[e] = e < rows * Nc ? xv[e] : make_double2(0.0, 0.0);
        __syncthreads();
        if (NP <= 256) {
            const int pair = t % NP, g = t / NP;
            const int c = pair / Nmu, mu = pair - c * Nmu;
            double2 acc = make_double2(0.0, 0.0);
            if (g < G)
                for (int r = g; r < rows; r += G) acc = cadd(acc, cmul(sA[r * Nmu + mu], sX[r * Nc + c]));
            red[t] = acc;
            __syncthreads();
            if (t < NP) {
                double2 sum = red[t];
                for (int gg = 1; gg < G; ++gg) sum = cadd(sum, red[gg * NP + t]);
                part[((size_t)blockIdx.x * nv + v) * NP + t] = sum;
            }
        } else {
            for (int pair = t; pair < NP; pair += 256) {
                const int c = pair / Nmu, mu = pair - c * Nmu;
                double2 acc = make_double2(0.0, 0.0);
                for (int r = 0; r < rows; ++r) acc = cadd(acc, cmul(sA[r * Nmu + mu], sX[r * Nc + c]));
                part[((size_t)blockIdx.x * nv + v) * NP + pair] = acc;
            }
        }
        __syncthreads();
    }
}

// b = sum over blocks (group g of pair p adds blocks g, g + G, ... in that order, eight loads
// in flight at a time; then the groups in order); b' = K b
__global__ __launch_bounds__(1024) void local_mat_kernel(const double2* __restrict__ part,
                                                         const double2* __restrict__ K,
                                                         double2* __restrict__ bprime, int nv,
                                                         int NP, int nblk) {
    __shared__ double2 red[1024];
    __shared__ double2 bsh[kMaxPairs];
    const int v = blockIdx.x;
    const int t = threadIdx.x;
    const int G = 1024 / NP;
    const int p = t % NP, g = t / NP;
    double2 s = make_double2(0.0, 0.0);
    if (g < G) {
        for (int b0 = g; b0 < nblk; b0 += 8 * G) {
            double2 q[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int b = b0 + u * G;
                q[u] = b < nblk ? part[((size_t)b * nv + v) * NP + p] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (b0 + u * G < nblk) s = cadd(s, q[u]);
        }
    }
    red[t] = s;
    __syncthreads();
    if (t < NP) {
        double2 sum = red[t];
        for (int gg = 1; gg < G; ++gg) sum = cadd(sum, red[gg * NP + t]);
        bsh[t] = sum;
    }
    __syncthreads();
    if (t < NP) {
        double2 o = make_double2(0.0, 0.0);
        for (int qq = 0; qq < NP; ++qq) o = cadd(o, cmul(K[(size_t)t * NP + qq], bsh[qq]));
        bprime[(size_t)v * NP + t] = o;
    }
}

// ---- combine: y = E x + Hc x + conj(A) b' - sum_s part[s] -----------------------------------------
// One thread per element (k, n, c) of vector v = blockIdx.y; block b covers elements
// [b per, (b + 1) per) of that vector, so each vector's dot partials are contiguous.  The
// back-projection partials of the S x chunks are added in chunk order.  Optionally also the
// block partial of Re<x|y> for Lanczos.
__global__ __launch_bounds__(256) void combine_kernel(
    const double2* __restrict__ x, double2* __restrict__ y, const double* __restrict__ E,
    const double2* __restrict__ Hc, const double2* __restrict__ A, const double2* __restrict__ bprime,
    const double2* __restrict__ part, int S, int nv, long long NkNb, int Nc, int Nmu, int has_core,
    double* __restrict__ dot_part, long long per_block) {
    __shared__ double sh[256];
    __shared__ double2 sHc[kMaxCore * kMaxCore];
    __shared__ double2 sB[kMaxPairs];
    const int cols = nv * Nc;
    const int v = blockIdx.y;
    for (int e = threadIdx.x; e < Nc * Nc; e += blockDim.x) sHc[e] = has_core ? Hc[e] : make_double2(0.0, 0.0);
    for (int e = threadIdx.x; e < Nc * Nmu; e += blockDim.x) sB[e] = bprime[(size_t)v * Nc * Nmu + e];
    __syncthreads();
    const long long n_el = NkNb * Nc;
    const long long start = (long long)blockIdx.x * per_block;
    const long long stop = min(n_el, start + per_block);
    const double2* xv = x + (size_t)v * n_el;
    double dot = 0.0;
    for (long long e = start + threadIdx.x; e < stop; e += blockDim.x) {
        const long long kn = e / Nc;
        const int c = (int)(e - kn * Nc);
        const double2 xe = xv[e];
        const double en = E[kn];
        double2 acc = make_double2(en * xe.x, en * xe.y);
        if (has_core) {
            const double2* xrow = xv + kn * Nc;
            for (int d = 0; d < Nc; ++d) acc = cadd(acc, cmul(sHc[c * Nc + d], xrow[d]));
        }
        for (int mu = 0; mu < Nmu; ++mu) acc = cadd(acc, cmulc(A[kn * Nmu + mu], sB[c * Nmu + mu]));
        double2 w0 = make_double2(0.0, 0.0);
        for (int sc = 0; sc < S; ++sc) w0 = cadd(w0, part[((size_t)sc * NkNb + kn) * cols + v * Nc + c]);
        acc.x -= w0.x;
        acc.y -= w0.y;
        y[(size_t)v * n_el + e] = acc;
        dot += xe.x * acc.x + xe.y * acc.y;
    }
    if (dot_part != nullptr) {
        const double s = block_sum(dot, sh);
        if (threadIdx.x == 0) dot_part[(size_t)v * gridDim.x + blockIdx.x] = s;
    }
}

// ---- Lanczos ------------------------------------------------------------------------------------------
// Vectors are [v][dim] complex; block b of vector v covers [b*per, (b+1)*per).

__global__ __launch_bounds__(256) void lz_norm_partial_kernel(const double2* __restrict__ p,
                                                              double* __restrict__ part,
                                                              long long dim, long long per) {
    __shared__ double sh[256];
    const int v = blockIdx.y;
    const double2* pv = p + (size_t)v * dim;
    const long long s0 = (long long)blockIdx.x * per, s1 = min(dim, s0 + per);
    double acc = 0.0;
    for (long long e = s0 + threadIdx.x; e < s1; e += blockDim.x) acc += pv[e].x * pv[e].x + pv[e].y * pv[e].y;
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[(size_t)v * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void lz_dot_partial_kernel(const double2* __restrict__ a,
                                                             const double2* __restrict__ b,
                                                             double* __restrict__ part,
                                                             long long dim, long long per) {
    __shared__ double sh[256];
    const int v = blockIdx.y;
    const double2* av = a + (size_t)v * dim;
    const double2* bv = b + (size_t)v * dim;
    const long long s0 = (long long)blockIdx.x * per, s1 = min(dim, s0 + per);
    double acc = 0.0;
    for (long long e = s0 + threadIdx.x; e < s1; e += blockDim.x) acc += av[e].x * bv[e].x + av[e].y * bv[e].y;
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[(size_t)v * gridDim.x + blockIdx.x] = s;
}

// Sum of nblk <= 256 block partials, computed by every lane of the calling wave (all 64 lanes
// must be active): lane l adds part[l], part[l + 64], ... in order, then a fixed xor-shuffle
// tree combines the lanes.  Every wave and every run gets the same bits.
static_assert(kRedBlocks <= 256, "sum_parts reads at most 256 partials");
__device__ __forceinline__ double sum_parts(const double* part, int nblk) {
    const int l = threadIdx.x & 63;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (l + 64 * u < nblk) s += part[l + 64 * u];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

// v = psi0 / |psi0|, vprev = 0, state reset; basis[0] = v when reorthogonalising
__global__ __launch_bounds__(256) void lz_init_kernel(const double2* __restrict__ psi0,
                                                      double2* __restrict__ vcur,
                                                      double2* __restrict__ vprev,
                                                      double2* __restrict__ basis,
                                                      const double* __restrict__ part,
                                                      LzState* __restrict__ st, int* __restrict__ step,
                                                      long long dim, long long per, int nstore) {
    const int v = blockIdx.y;
    const double n2 = sum_parts(part + (size_t)v * gridDim.x, gridDim.x);
    const double inv = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
    const long long s0 = (long long)blockIdx.x * per, s1 = min(dim, s0 + per);
    for (long long e = s0 + threadIdx.x; e < s1; e += blockDim.x) {
        const double2 p = psi0[(size_t)v * dim + e];
        const double2 q = make_double2(p.x * inv, p.y * inv);
        vcur[(size_t)v * dim + e] = q;
        vprev[(size_t)v * dim + e] = make_double2(0.0, 0.0);
        if (basis) basis[(size_t)v * nstore * dim + e] = q;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        LzState s;
        s.b_cur = 0.0;
        s.scale = 0.0;
        s.norm2 = n2;
        s.a_cur = 0.0;
        s.done = n2 > 0.0 ? 0 : 1;
        s.steps = 0;
        s.pad[0] = s.pad[1] = 0;
        st[v] = s;
        if (v == 0) *step = 0;
    }
}

// a_i = sum of partials; w -= a_i v + b_i vprev; optional |w|^2 partials; block 0 records a_i
__global__ __launch_bounds__(256) void lz_update_kernel(double2* __restrict__ w,
                                                        const double2* __restrict__ vcur,
                                                        const double2* __restrict__ vprev,
                                                        const double* __restrict__ part_a,
                                                        double* __restrict__ part_n,
                                                        LzState* __restrict__ st,
                                                        double* __restrict__ a_out,
                                                        const int* __restrict__ step,
                                                        int n_steps, long long dim, long long per,
                                                        int nblk_a) {
    __shared__ double sh[256];
    const int v = blockIdx.y;
    const int i = *step;
    const double a = sum_parts(part_a + (size_t)v * nblk_a, nblk_a);
    const double bi = st[v].b_cur;
    const bool done = st[v].done != 0;
    const long long s0 = (long long)blockIdx.x * per, s1 = min(dim, s0 + per);
    double acc = 0.0;
    for (long long e = s0 + threadIdx.x; e < s1; e += blockDim.x) {
        const size_t o = (size_t)v * dim + e;
        double2 ww = w[o];
        if (!done) {
            const double2 vc = vcur[o], vp = vprev[o];
            ww.x = ww.x - a * vc.x - bi * vp.x;
            ww.y = ww.y - a * vc.y - bi * vp.y;
            w[o] = ww;
        }
        acc += ww.x * ww.x + ww.y * ww.y;
    }
    if (part_n != nullptr) {
        const double s = block_sum(acc, sh);
        if (threadIdx.x == 0) part_n[(size_t)v * gridDim.x + blockIdx.x] = s;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && !done) {
        a_out[(size_t)v * n_steps + i] = a;
        st[v].a_cur = a;
    }
}

// Re-orthogonalisation, pass 1: hpart[v][b][j] = sum_{e in block b} conj(basis_j[e]) w[e], j <= step
__global__ __launch_bounds__(256) void lz_reorth_dot_kernel(const double2* __restrict__ basis,
                                                            const double2* __restrict__ w,
                                                            double2* __restrict__ hpart,
                                                            const LzState* __restrict__ st,
                                                            const int* __restrict__ step,
                                                            long long dim, long long per,
                                                            int nstore) {
    __shared__ double sh[256];
    const int v = blockIdx.y;
    if (st[v].done) return;
    const int nj = *step + 1;
    const long long s0 = (long long)blockIdx.x * per, s1 = min(dim, s0 + per);
    const double2* wv = w + (size_t)v * dim;
    for (int j = 0; j < nj; ++j) {
        const double2* bj = basis + ((size_t)v * nstore + j) * dim;
        double2 acc = make_double2(0.0, 0.0);
        for (long long e = s0 + threadIdx.x; e < s1; e += blockDim.x) acc = cadd(acc, cmulc(bj[e], wv[e]));
        const double2 s = block_sum2(acc, sh);
        if (threadIdx.x == 0) hpart[((size_t)v * gridDim.x + blockIdx.x) * nstore + j] = s;
    }
}

// pass 2: h_j = sum over blocks (fixed order)
__global__ __launch_bounds__(256) void lz_reorth_fin_kernel(const double2* __restrict__ hpart,
                                                            double2* __restrict__ hcoef,
                                                            const LzState* __restrict__ st,
                                                            const int* __restrict__ step,
                                                            int nblk, int nstore) {
    const int v = blockIdx.x;
    if (st[v].done) return;
    const int nj = *step + 1;
    for (int j = threadIdx.x; j < nj; j += blockDim.x) {
        double2 s = make_double2(0.0, 0.0);
        for (int b = 0; b < nblk; ++b) s = cadd(s, hpart[((size_t)v * nblk + b) * nstore + j]);
        hcoef[(size_t)v * nstore + j] = s;
    }
}

// pass 3: w -= sum_j h_j basis_j
__global__ __launch_bounds__(256) void lz_reorth_sub_kernel(const double2* __restrict__ basis,
                                                            double2* __restrict__ w,
                                                            const double2* __restrict__ hcoef,
                                                            const LzState* __restrict__ st,
                                                            const int* __restrict__ step,
                                                            long long dim, long long per,
                                                            int nstore) {
    const int v = blockIdx.y;
    if (st[v].done) return;
    const int nj = *step + 1;
    const long long s0 = (long long)blockIdx.x * per, s1 = min(dim, s0 + per);
    for (long long e = s0 + threadIdx.x; e < s1; e += blockDim.x) {
        double2 acc = make_double2(0.0, 0.0);
        for (int j = 0; j < nj; ++j)
            acc = cadd(acc, cmul(hcoef[(size_t)v * nstore + j], basis[((size_t)v * nstore + j) * dim + e]));
        const size_t o = (size_t)v * dim + e;
        w[o] = make_double2(w[o].x - acc.x, w[o].y - acc.y);
    }
}

// b_{i+1} = sqrt(sum |w|^2 partials); breakdown test; record b
__global__ __launch_bounds__(64) void lz_finalize_kernel(const double* __restrict__ part_n,
                                                         LzState* __restrict__ st,
                                                         double* __restrict__ b_out,
                                                         const int* __restrict__ step, int n_steps,
                                                         int nblk) {
    const int v = blockIdx.x;
    const double b2 = sum_parts(part_n + (size_t)v * nblk, nblk);  // the whole wave
    if (threadIdx.x != 0) return;
    LzState s = st[v];
    if (s.done) return;
    const int i = *step;
    const double b = sqrt(b2);
    s.scale = fmax(s.scale, fmax(fabs(s.a_cur), s.b_cur));
    b_out[(size_t)v * n_steps + i] = b;
    s.steps = i + 1;
    if (b <= 1e-14 * s.scale) s.done = 1;
    s.b_cur = b;
    st[v] = s;
}

// vprev = v; v = w / b_{i+1}; basis[i+1] = v
__global__ __launch_bounds__(256) void lz_scale_kernel(const double2* __restrict__ w,
                                                       double2* __restrict__ vcur,
                                                       double2* __restrict__ vprev,
                                                       double2* __restrict__ basis,
                                                       const LzState* __restrict__ st,
                                                       const int* __restrict__ step, long long dim,
                                                       long long per, int nstore) {
    const int v = blockIdx.y;
    if (st[v].done) return;
    const double inv = 1.0 / st[v].b_cur;
    const int i = *step;
    const long long s0 = (long long)blockIdx.x * per, s1 = min(dim, s0 + per);
    for (long long e = s0 + threadIdx.x; e < s1; e += blockDim.x) {
        const size_t o = (size_t)v * dim + e;
        const double2 ww = w[o];
        const double2 q = make_double2(ww.x * inv, ww.y * inv);
        vprev[o] = vcur[o];
        vcur[o] = q;
        if (basis && i + 1 < nstore) basis[((size_t)v * nstore + i + 1) * dim + e] = q;
    }
}

__global__ void lz_advance_kernel(int* step) { *step += 1; }

// ---- continued fraction -------------------------------------------------------------------------------
__device__ __forceinline__ double2 cdiv1(double2 z) {  // 1 / z
    const double d = z.x * z.x + z.y * z.y;
    return make_double2(z.x / d, -z.y / d);
}

__device__ double2 csqrt_principal(double2 w) {
    const double r = sqrt(w.x * w.x + w.y * w.y);
    if (r == 0.0) return make_double2(0.0, 0.0);
    const double s = sqrt(0.5 * (r + fabs(w.x)));
    if (w.x >= 0.0) return make_double2(s, w.y / (2.0 * s));
    return make_double2(fabs(w.y) / (2.0 * s), copysign(s, w.y));
}

__global__ __launch_bounds__(256) void spectrum_kernel(const double* __restrict__ a,
                                                       const double* __restrict__ b,
                                                       const int* __restrict__ n_used,
                                                       const double* __restrict__ norm2,
                                                       int n_spec, int n_steps, int terminator,
                                                       const double* __restrict__ a_inf,
                                                       const double* __restrict__ b_inf,
                                                       const double* __restrict__ omega,
                                                       int n_omega, double gamma,
                                                       double* __restrict__ sigma) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n_spec * n_omega) return;
    const int sp = (int)(idx / n_omega), o = (int)(idx - (long long)sp * n_omega);
    const double* as = a + (size_t)sp * n_steps;
    const double* bs = b + (size_t)sp * n_steps;
    const int N = n_used ? n_used[sp] : n_steps;
    const double2 z = make_double2(omega[o], gamma);
    double2 g = make_double2(0.0, 0.0);
    if (terminator == OCEAN_TERM_SQRT && N > 0) {
        double ai = 0.0, bi = 0.0;
        if (a_inf) {
            ai = a_inf[sp];
            bi = b_inf[sp];
        } else {
            const int tail = N < 16 ? N : 16;
            for (int j = N - tail; j < N; ++j) {
                ai += as[j];
                bi += bs[j];
            }
            ai /= tail;
            bi /= tail;
        }
        const double2 zz = make_double2(z.x - ai, z.y);
        const double2 disc = make_double2(zz.x * zz.x - zz.y * zz.y - 4.0 * bi * bi, 2.0 * zz.x * zz.y);
        const double2 sq = csqrt_principal(disc);
        const double den = 2.0 * bi * bi;
        const double2 t1 = make_double2((zz.x - sq.x) / den, (zz.y - sq.y) / den);
        const double2 t2 = make_double2((zz.x + sq.x) / den, (zz.y + sq.y) / den);
        g = t1.y <= 0.0 ? t1 : t2;
    }
    for (int i = N - 1; i >= 0; --i) {
        const double bb = bs[i] * bs[i];
        const double2 den = make_double2(z.x - as[i] - bb * g.x, z.y - bb * g.y);
        g = cdiv1(den);
    }
    sigma[idx] = -norm2[sp] * g.y * 0.31830988618379067154;  // 1/pi
}

// ---- set-up kernels ---------------------------------------------------------------------------------------
// W[x][R] = W_rad(|minimum image of x + R - tau|), linear interpolation of the radial table
__global__ __launch_bounds__(256) void build_w_kernel(double* __restrict__ W64, float* __restrict__ W32,
                                                      const double* __restrict__ wr,
                                                      const double* __restrict__ wv, int n_wr,
                                                      double hstep, int n1, int n2, int n3,
                                                      int g1, int g2, int g3, WGeom geo) {
    const long long Nk = (long long)n1 * n2 * n3;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long Nx = (long long)g1 * g2 * g3;
    if (idx >= Nx * Nk) return;
    // layout [x][R2 R3][R1]: R1 fastest, so the k1 pass of the transform reads one pencil
    // of W as a contiguous vector
    const int x = (int)(idx / Nk), q = (int)(idx - (long long)x * Nk);
    const int j3 = x % g3, j2 = (x / g3) % g2, j1 = x / (g2 * g3);
    const int r1 = q % n1, r23 = q / n1;
    const int r3 = r23 % n3, r2 = r23 / n3;
    // x + R - tau in cartesian coordinates (fractional cell coordinates times the rows a_d)
    const double c[3] = {(double)j1 / g1 + r1, (double)j2 / g2 + r2, (double)j3 / g3 + r3};
    double d[3];
    for (int b = 0; b < 3; ++b) d[b] = c[0] * geo.A[b] + c[1] * geo.A[3 + b] + c[2] * geo.A[6 + b] - geo.tau[b];
    // fractional coordinates in the supercell (rows S_d = n_d a_d), wrapped into [-1/2, 1/2]
    double f[3];
    for (int a = 0; a < 3; ++a) {
        f[a] = d[0] * geo.Sinv[a] + d[1] * geo.Sinv[3 + a] + d[2] * geo.Sinv[6 + a];
        f[a] -= rint(f[a]);
    }
    // nearest image: the wrapped point itself for mutually orthogonal S_d, else the nearest
    // of the 27 translations around it
    double dist2 = 1e300;
    const int reach = geo.ortho ? 0 : 1;
    for (int m0 = -reach; m0 <= reach; ++m0)
        for (int m1 = -reach; m1 <= reach; ++m1)
            for (int m2 = -reach; m2 <= reach; ++m2) {
                const double e0 = f[0] + m0, e1 = f[1] + m1, e2 = f[2] + m2;
                double s2 = 0.0;
                for (int b = 0; b < 3; ++b) {
                    const double v = e0 * geo.S[b] + e1 * geo.S[3 + b] + e2 * geo.S[6 + b];
                    s2 += v * v;
                }
                dist2 = fmin(dist2, s2);
            }
    const double dist = sqrt(dist2);
    const double rmax = wr[n_wr - 1];
    double val;
    if (dist >= rmax) {
        val = wv[n_wr - 1] * rmax / dist;
    } else {
        const double s = dist / hstep;
        int j = (int)floor(s);
        if (j > n_wr - 2) j = n_wr - 2;
        const double t = s - j;
        val = (1.0 - t) * wv[j] + t * wv[j + 1];
    }
    // the 1/Nk of the unitary k <-> R pair is folded into the table
    val /= (double)Nk;
    if (W64) W64[idx] = val;
    if (W32) W32[idx] = (float)val;
}

// rows g0 .. g0 + rows - 1 of u (row g = k Nx + x, Nb complex FP64 each) times their Bloch
// phase, stored as T (FP64 in place is allowed: each element is read before it is written)
template <typename T>
__global__ __launch_bounds__(256) void u_phase_kernel(const double* __restrict__ src, long long g0, long long rows,
                                                     int Nb, PhaseArgs pa, T* dst) {
    const long long n_el = rows * Nb;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n_el; e += stride) {
        const double2 ph = bloch_phase(pa, g0 + e / Nb);
        const double re = src[2 * e], im = src[2 * e + 1];
        dst[2 * e] = (T)(re * ph.x - im * ph.y);
        dst[2 * e + 1] = (T)(re * ph.y + im * ph.x);
    }
}

// psi0[p][kn][(mc, s)] = sum_m conj(A[kn][m]) d_p[m][mc]
// Nc = 6: core index (m_c, sigma), the same amplitude for both spins.  Nc = 12 (electron spin
// carried separately): index ((m_c, sigma_h), sigma_e), amplitude on sigma_e = sigma_h only,
// since the dipole operator does not flip the spin.
__global__ __launch_bounds__(256) void dipole_kernel(const double2* __restrict__ A,
                                                     const double2* __restrict__ d,
                                                     double2* __restrict__ psi0, int n_pol,
                                                     long long NkNb, int Nc, int Nmu) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n_pol * NkNb) return;
    const int p = (int)(idx / NkNb);
    const long long kn = idx - (long long)p * NkNb;
    const double2* dp = d + (size_t)p * Nmu * 3;   // [mu][m_c] amplitudes of polarisation p
    for (int mc = 0; mc < 3; ++mc) {
        double2 acc = make_double2(0.0, 0.0);
        for (int m = 0; m < Nmu; ++m) acc = cadd(acc, cmulc(A[kn * Nmu + m], dp[m * 3 + mc]));
        if (Nc == 6) {
            psi0[idx * 6 + mc * 2 + 0] = acc;
            psi0[idx * 6 + mc * 2 + 1] = acc;
        } else {
            for (int s = 0; s < 2; ++s)
                for (int e = 0; e < 2; ++e)
                    psi0[idx * 12 + (mc * 2 + s) * 2 + e] = s == e ? acc : make_double2(0.0, 0.0);
        }
    }
}

// w0[kn][col] = sum over chunks s of part[s][kn][col].  A block of 256 threads sums 256 / G
// elements: element e = blockIdx.x * (256 / G) + t % (256 / G) is summed by G threads over
// s = g, g + G, ... (g = t / (256 / G)), and the G partial sums are then added in the order
// g = 0, 1, ...  G = 4 for a few chunks; G = 16 when there are many (Gamma-only systems with
// large grids), so that more blocks share the work and each thread walks fewer chunks.
template <int G>
__global__ __launch_bounds__(256) void reduce_part_kernel(const double2* __restrict__ part,
                                                         double2* __restrict__ w0, int S,
                                                         long long n_elem) {
    constexpr int EB = 256 / G;   // elements per block
    __shared__ double2 sh[256];
    const int t = threadIdx.x;
    const int g = t / EB;
    const long long e = (long long)blockIdx.x * EB + (t % EB);
    double2 acc = make_double2(0.0, 0.0);
    if (e < n_elem)
        for (int s = g; s < S; s += G) acc = cadd(acc, part[(size_t)s * n_elem + e]);
    sh[t] = acc;
    __syncthreads();
    if (g == 0 && e < n_elem) {
        double2 r = sh[t];
#pragma unroll
        for (int j = 1; j < G; ++j) r = cadd(r, sh[t + j * EB]);
        w0[e] = r;
    }
}

// Gamma-point-only grids: the k-grid transform is the identity and W(x, R = 0) is diagonal
// in x, so the transform and W steps of Algorithm 1 reduce to phi[x][col] *= W[x].
// C2: compute type, S: stored type of phi
template <typename C2, typename S, typename T>
__global__ __launch_bounds__(256) void w_gamma_kernel(S* __restrict__ phi, const T* __restrict__ W,
                                                     long long n_elem, int cols) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem; e += stride) {
        const T w = W[e / cols];
        C2 v = phi_load<C2>(&phi[e]);
        v.x *= w;
        v.y *= w;
        phi_store(&phi[e], v);
    }
}

inline long long per_block(long long dim) { return (dim + kRedBlocks - 1) / kRedBlocks; }

}  // namespace

// ---- launchers ---------------------------------------------------------------------------------------------
long long local_blocks(const ocean_bse_s* h) {
    const long long NkNb = (long long)h->Nk * h->Nb;
    const int R = local_rows(h->Nc, h->Nmu);
    return (NkNb + R - 1) / R;
}

hipError_t launch_local_in(ocean_bse_s* h, const double* x, int nv) {
    const long long NkNb = (long long)h->Nk * h->Nb;
    const long long nblk = local_blocks(h);
    const int slot = prof_begin(h, "local_in");
    const int R = local_rows(h->Nc, h->Nmu);
    local_in_kernel<<<(unsigned)nblk, 256, (size_t)R * (h->Nmu + h->Nc) * sizeof(double2), h->stream>>>(
        reinterpret_cast<const double2*>(x), reinterpret_cast<const double2*>(h->A),
        reinterpret_cast<double2*>(h->ws.loc_part), nv, NkNb, h->Nc, h->Nmu, R);
    prof_end(h, slot);
    return hipGetLastError();
}

hipError_t launch_local_mat(ocean_bse_s* h, int nv) {
    const int slot = prof_begin(h, "local_mat");
    local_mat_kernel<<<nv, 1024, 0, h->stream>>>(reinterpret_cast<const double2*>(h->ws.loc_part),
                                                reinterpret_cast<const double2*>(h->K),
                                                reinterpret_cast<double2*>(h->ws.loc_b), nv,
                                                h->Nc * h->Nmu, (int)local_blocks(h));
    prof_end(h, slot);
    return hipGetLastError();
}

hipError_t launch_reduce_part(ocean_bse_s* h, int nv) {
    const long long n_elem = (long long)h->Nk * h->Nb * nv * h->Nc;
    const int slot = prof_begin(h, "reduce_part");
    const double2* part = reinterpret_cast<const double2*>(h->ws.part);
    double2* w0 = reinterpret_cast<double2*>(h->ws.w0);
    if (h->ws.bwd_chunks > 16)
        reduce_part_kernel<16><<<(unsigned)((n_elem + 15) / 16), 256, 0, h->stream>>>(part, w0, h->ws.bwd_chunks,
                                                                                    n_elem);
    else
        reduce_part_kernel<4><<<(unsigned)((n_elem + 63) / 64), 256, 0, h->stream>>>(part, w0, h->ws.bwd_chunks,
                                                                                  n_elem);
    prof_end(h, slot);
    return hipGetLastError();
}

hipError_t launch_w_gamma(ocean_bse_s* h, int cols) {
    const long long n_elem = (long long)h->Nx * cols;
    const unsigned nblk = (unsigned)std::min<long long>((n_elem + 255) / 256, 65536);
    const int slot = prof_begin(h, "fft_w");
    if (h->precision == OCEAN_PREC_FP64)
        w_gamma_kernel<double2, double2, double><<<nblk, 256, 0, h->stream>>>(static_cast<double2*>(h->ws.phi), h->W64, n_elem, cols);
    else if (h->precision == OCEAN_PREC_BF16)
        w_gamma_kernel<float2, bf16c, float><<<nblk, 256, 0, h->stream>>>(static_cast<bf16c*>(h->ws.phi), h->W32, n_elem, cols);
    else
        w_gamma_kernel<float2, float2, float><<<nblk, 256, 0, h->stream>>>(static_cast<float2*>(h->ws.phi), h->W32, n_elem, cols);
    prof_end(h, slot);
    return hipGetLastError();
}

hipError_t launch_combine(ocean_bse_s* h, const double* x, double* y, int nv, double* dot_part) {
    const long long n_el = (long long)h->Nk * h->Nb * h->Nc;
    const long long per = (n_el + kRedBlocks - 1) / kRedBlocks;
    dim3 grid(kRedBlocks, nv);
    // few x chunks: read the back-projection partials here; many: from their sum
    const bool direct = h->ws.bwd_chunks <= kCombineDirectChunks;
    const int slot = prof_begin(h, "combine");
    combine_kernel<<<grid, 256, 0, h->stream>>>(
        reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), h->E,
        reinterpret_cast<const double2*>(h->Hc), reinterpret_cast<const double2*>(h->A),
        reinterpret_cast<const double2*>(h->ws.loc_b),
        reinterpret_cast<const double2*>(direct ? h->ws.part : h->ws.w0), direct ? h->ws.bwd_chunks : 1, nv,
        (long long)h->Nk * h->Nb, h->Nc, h->Nmu > 0 && h->K != nullptr ? h->Nmu : 0, h->Hc != nullptr, dot_part, per);
    prof_end(h, slot);
    return hipGetLastError();
}

hipError_t lz_init(ocean_bse_s* h, const double* psi0, int nv) {
    const long long dim = (long long)h->Nk * h->Nb * h->Nc;
    const long long per = per_block(dim);
    dim3 grid(kRedBlocks, nv);
    auto& L = h->lz;
    const int nstore = L.n_steps + 1;
    int slot = prof_begin(h, "lz_norm");
    lz_norm_partial_kernel<<<grid, 256, 0, h->stream>>>(reinterpret_cast<const double2*>(psi0),
                                                        L.part_n, dim, per);
    prof_end(h, slot);
    slot = prof_begin(h, "lz_init");
    lz_init_kernel<<<grid, 256, 0, h->stream>>>(
        reinterpret_cast<const double2*>(psi0), reinterpret_cast<double2*>(L.v),
        reinterpret_cast<double2*>(L.vprev), reinterpret_cast<double2*>(L.basis), L.part_n,
        L.state, L.step, dim, per, nstore);
    prof_end(h, slot);
    return hipGetLastError();
}

hipError_t lz_dot_vw(ocean_bse_s* h, int nv) {
    const long long dim = (long long)h->Nk * h->Nb * h->Nc;
    dim3 grid(kRedBlocks, nv);
    const int slot = prof_begin(h, "lz_dot");
    lz_dot_partial_kernel<<<grid, 256, 0, h->stream>>>(reinterpret_cast<const double2*>(h->lz.v),
                                                       reinterpret_cast<const double2*>(h->lz.w),
                                                       h->lz.part_a, dim, per_block(dim));
    prof_end(h, slot);
    return hipGetLastError();
}

hipError_t lz_update(ocean_bse_s* h, int nv, bool with_norm) {
    const long long dim = (long long)h->Nk * h->Nb * h->Nc;
    dim3 grid(kRedBlocks, nv);
    auto& L = h->lz;
    const int slot = prof_begin(h, "lz_update");
    lz_update_kernel<<<grid, 256, 0, h->stream>>>(
        reinterpret_cast<double2*>(L.w), reinterpret_cast<const double2*>(L.v),
        reinterpret_cast<const double2*>(L.vprev), L.part_a, with_norm ? L.part_n : nullptr,
        L.state, L.a, L.step, L.n_steps, dim, per_block(dim), kRedBlocks);
    prof_end(h, slot);
    return hipGetLastError();
}

hipError_t lz_reorth(ocean_bse_s* h, int nv) {
    const long long dim = (long long)h->Nk * h->Nb * h->Nc;
    dim3 grid(kRedBlocks, nv);
    auto& L = h->lz;
    const int nstore = L.n_steps + 1;
    const int slot = prof_begin(h, "lz_reorth");
    for (int pass = 0; pass < 2; ++pass) {
        lz_reorth_dot_kernel<<<grid, 256, 0, h->stream>>>(
            reinterpret_cast<const double2*>(L.basis), reinterpret_cast<const double2*>(L.w),
            reinterpret_cast<double2*>(L.hpart), L.state, L.step, dim, per_block(dim), nstore);
        lz_reorth_fin_kernel<<<nv, 256, 0, h->stream>>>(reinterpret_cast<const double2*>(L.hpart),
                                                        reinterpret_cast<double2*>(L.hcoef),
                                                        L.state, L.step, kRedBlocks, nstore);
        lz_reorth_sub_kernel<<<grid, 256, 0, h->stream>>>(
            reinterpret_cast<const double2*>(L.basis), reinterpret_cast<double2*>(L.w),
            reinterpret_cast<const double2*>(L.hcoef), L.state, L.step, dim, per_block(dim), nstore);
    }
    prof_end(h, slot);
    return hipGetLastError();
}

hipError_t lz_norm_w(ocean_bse_s* h, int nv) {
    const long long dim = (long long)h->Nk * h->Nb * h->Nc;
    dim3 grid(kRedBlocks, nv);
    const int slot = prof_begin(h, "lz_norm");
    lz_norm_partial_kernel<<<grid, 256, 0, h->stream>>>(reinterpret_cast<const double2*>(h->lz.w),
                                                        h->lz.part_n, dim, per_block(dim));
    prof_end(h, slot);
    return hipGetLastError();
}

hipError_t lz_finalize(ocean_bse_s* h, int nv) {
    const int slot = prof_begin(h, "lz_finalize");
    lz_finalize_kernel<<<nv, 64, 0, h->stream>>>(h->lz.part_n, h->lz.state, h->lz.b, h->lz.step,
                                                 h->lz.n_steps, kRedBlocks);
    prof_end(h, slot);
    return hipGetLastError();
}

hipError_t lz_scale(ocean_bse_s* h, int nv) {
    const long long dim = (long long)h->Nk * h->Nb * h->Nc;
    dim3 grid(kRedBlocks, nv);
    auto& L = h->lz;
    const int slot = prof_begin(h, "lz_scale");
    lz_scale_kernel<<<grid, 256, 0, h->stream>>>(
        reinterpret_cast<const double2*>(L.w), reinterpret_cast<double2*>(L.v),
        reinterpret_cast<double2*>(L.vprev), reinterpret_cast<double2*>(L.basis), L.state, L.step,
        dim, per_block(dim), L.n_steps + 1);
    prof_end(h, slot);
    return hipGetLastError();
}

hipError_t lz_advance(ocean_bse_s* h) {
    lz_advance_kernel<<<1, 1, 0, h->stream>>>(h->lz.step);
    return hipGetLastError();
}

hipError_t launch_spectrum(const double* a, const double* b, const int* n_used, const double* norm2,
                           int n_spec, int n_steps, int terminator, const double* a_inf,
                           const double* b_inf, const double* omega,
                           int n_omega, double gamma, double* sigma, hipStream_t stream) {
    const long long n = (long long)n_spec * n_omega;
    spectrum_kernel<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(
        a, b, n_used, norm2, n_spec, n_steps, terminator, a_inf, b_inf, omega, n_omega, gamma, sigma);
    return hipGetLastError();
}

hipError_t launch_build_w(ocean_bse_s* h, const double* wr_dev, const double* wv_dev, int n_wr,
                          double h_r) {
    const long long n = (long long)h->Nx * h->Nk;
    WGeom geo;
    for (int i = 0; i < 9; ++i) {
        geo.A[i] = h->cell[i];
        geo.S[i] = h->cell[i] * h->nk[i / 3];
    }
    for (int b = 0; b < 3; ++b) geo.tau[b] = h->tau[b];
    // inverse of S by cofactors (S nonsingular: checked at creation)
    const double* S = geo.S;
    const double det = S[0] * (S[4] * S[8] - S[5] * S[7]) - S[1] * (S[3] * S[8] - S[5] * S[6]) +
                       S[2] * (S[3] * S[7] - S[4] * S[6]);
    geo.Sinv[0] = (S[4] * S[8] - S[5] * S[7]) / det;
    geo.Sinv[1] = (S[2] * S[7] - S[1] * S[8]) / det;
    geo.Sinv[2] = (S[1] * S[5] - S[2] * S[4]) / det;
    geo.Sinv[3] = (S[5] * S[6] - S[3] * S[8]) / det;
    geo.Sinv[4] = (S[0] * S[8] - S[2] * S[6]) / det;
    geo.Sinv[5] = (S[2] * S[3] - S[0] * S[5]) / det;
    geo.Sinv[6] = (S[3] * S[7] - S[4] * S[6]) / det;
    geo.Sinv[7] = (S[1] * S[6] - S[0] * S[7]) / det;
    geo.Sinv[8] = (S[0] * S[4] - S[1] * S[3]) / det;
    geo.ortho = 1;
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j) {
            double dot = 0.0, ni = 0.0, nj = 0.0;
            for (int b = 0; b < 3; ++b) {
                dot += S[3 * i + b] * S[3 * j + b];
                ni += S[3 * i + b] * S[3 * i + b];
                nj += S[3 * j + b] * S[3 * j + b];
            }
            if (std::fabs(dot) > 1e-12 * std::sqrt(ni * nj)) geo.ortho = 0;
        }
    build_w_kernel<<<(unsigned)((n + 255) / 256), 256, 0, h->stream>>>(
        h->W64, h->W32, wr_dev, wv_dev, n_wr, h_r, h->nk[0], h->nk[1], h->nk[2], h->nx[0],
        h->nx[1], h->nx[2], geo);
    return hipGetLastError();
}

PhaseArgs phase_args(const ocean_bse_s* h) {
    PhaseArgs p;
    p.ph = h->phase;
    for (int a = 0; a < 3; ++a) {
        p.po[a] = h->phase_off[a];
        p.nk[a] = h->nk[a];
        p.nx[a] = h->nx[a];
    }
    p.Nx = h->Nx;
    return p;
}

hipError_t launch_u_phase_fp64(ocean_bse_s* h, const double* src, long long g0, long long rows, double* dst) {
    u_phase_kernel<double><<<4096, 256, 0, h->stream>>>(src, g0, rows, h->Nb, phase_args(h), dst);
    return hipGetLastError();
}

hipError_t launch_u_to_fp32(ocean_bse_s* h, const double* src, long long g0, long long rows, float* dst) {
    u_phase_kernel<float><<<4096, 256, 0, h->stream>>>(src, g0, rows, h->Nb, phase_args(h), dst + 2 * g0 * h->Nb);
    return hipGetLastError();
}

hipError_t launch_dipole_psi0(ocean_bse_s* h, const double* d_dev, int n_pol, double* psi0) {
    const long long NkNb = (long long)h->Nk * h->Nb;
    const long long n = NkNb * n_pol;
    dipole_kernel<<<(unsigned)((n + 255) / 256), 256, 0, h->stream>>>(
        reinterpret_cast<const double2*>(h->A), reinterpret_cast<const double2*>(d_dev),
        reinterpret_cast<double2*>(psi0), n_pol, NkNb, h->Nc, h->Nmu);
    return hipGetLastError();
}

}  // namespace ocean
