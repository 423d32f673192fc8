// k-grid transform and screened-potential multiply of Algorithm 1 lines 3-5
// (section 3.2.1), with the e^{+-ik.x} phases of lines 2 and 6 folded in:
//
//   phi(x, R)  = Nk^{-1/2} sum_k e^{+ik.R} e^{+ik.x} phi(x, k)      (line 3)
//   phi(x, R) *= W(x, R)                                            (line 4)
//   phi'(x, k) = Nk^{-1/2} e^{-ik.x} sum_R e^{-ik.R} phi(x, R)       (line 5)
//
// A line is one (x, column) pair; its Nk values sit at stride Nx*cols in
// phi[k][x][col].  A block stages L consecutive lines (contiguous for every k)
// in LDS as [k][line], runs the separable small DFTs along the three k axes in
// LDS, multiplies by W and transforms back, then writes the lines in place.
// W(x, R) is stored [x][R2 R3][R1] (R1 fastest), R = R1 n2 n3 + R2 n3 + R3.
// The pass is HBM-bound: phi is read once and written once.
#include "internal.h"

namespace ocean {
namespace {

template <typename T> struct C2T;
template <> struct C2T<double> { typedef double2 t; };
template <> struct C2T<float> { typedef float2 t; };

// N consecutive W values, aligned to their size so that they load as wide vectors
template <typename T, int N> struct alignas(sizeof(T) * N) WVec { T v[N]; };

template <typename C2> __device__ __forceinline__ C2 cmul(C2 a, C2 b) {
    C2 r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

// One pass of length-n DFTs (n <= NMAX) along an axis of stride `st` (in k units).
template <typename T, int NMAX>
__device__ __forceinline__ void dft_pass(typename C2T<T>::t* buf, const typename C2T<T>::t* tw,
                                         int n, int st, int Nk, int L, bool inverse) {
    typedef typename C2T<T>::t C2;
    const int ntr = (Nk / n) * L;
    for (int idx = threadIdx.x; idx < ntr; idx += blockDim.x) {
        const int l = idx % L;
        const int u = idx / L;
        const int base = (u / st) * (n * st) + (u % st);
        C2 in[NMAX];
#pragma unroll
        for (int b = 0; b < NMAX; ++b)
            if (b < n) in[b] = buf[(base + b * st) * L + l];
#pragma unroll
        for (int a = 0; a < NMAX; ++a) {
            if (a < n) {
                C2 acc;
                acc.x = 0;
                acc.y = 0;
#pragma unroll
                for (int b = 0; b < NMAX; ++b) {
                    if (b < n) {
                        C2 w = tw[(a * b) % n];
                        if (inverse) w.y = -w.y;
                        acc.x += in[b].x * w.x - in[b].y * w.y;
                        acc.y += in[b].x * w.y + in[b].y * w.x;
                    }
                }
                buf[(base + a * st) * L + l] = acc;
            }
        }
    }
}

template <typename T, int NMAX>
__device__ __forceinline__ void dft3(typename C2T<T>::t* buf, const typename C2T<T>::t* tw_lds,
                                     int n1, int n2, int n3, int L, bool inverse) {
    const int Nk = n1 * n2 * n3;
    if (n3 > 1) { dft_pass<T, NMAX>(buf, tw_lds + 2 * kMaxDft, n3, 1, Nk, L, inverse); __syncthreads(); }
    if (n2 > 1) { dft_pass<T, NMAX>(buf, tw_lds + 1 * kMaxDft, n2, n3, Nk, L, inverse); __syncthreads(); }
    if (n1 > 1) { dft_pass<T, NMAX>(buf, tw_lds, n1, n2 * n3, Nk, L, inverse); __syncthreads(); }
}

template <typename T, int NMAX>
__global__ __launch_bounds__(256) void fft_w_kernel(
    typename C2T<T>::t* __restrict__ phi, const T* __restrict__ W, const double2* __restrict__ ph,
    const double2* __restrict__ tw, int n1, int n2, int n3, int g1, int g2, int g3, int po1,
    int po2, int po3, int to1, int to2, int to3, int Nx, int cols, int L) {
    typedef typename C2T<T>::t C2;
    extern __shared__ __align__(16) unsigned char smem[];
    C2* tw_lds = reinterpret_cast<C2*>(smem);            // [3][kMaxDft]
    C2* buf = tw_lds + 3 * kMaxDft;                       // [Nk][L]
    const int Nk = n1 * n2 * n3;
    const long long total = (long long)Nx * cols;
    const long long line0 = (long long)blockIdx.x * L;
    const int nn[3] = {n1, n2, n3};
    const int to[3] = {to1, to2, to3};
    if (threadIdx.x < 3 * kMaxDft) {
        const int d = threadIdx.x / kMaxDft, m = threadIdx.x % kMaxDft;
        C2 v;
        v.x = 0;
        v.y = 0;
        if (m < nn[d]) {
            double2 t = tw[to[d] + m];
            v.x = (T)t.x;
            v.y = (T)t.y;
        }
        tw_lds[threadIdx.x] = v;
    }
    const T inv_nk = (T)(1.0 / (double)Nk);

    // load, with the e^{+ik.x} phase of line 2
    for (int e = threadIdx.x; e < Nk * L; e += blockDim.x) {
        const int kk = e / L, l = e - kk * L;
        const long long line = line0 + l;
        C2 v;
        v.x = 0;
        v.y = 0;
        if (line < total) {
            v = phi[phi_index(line, kk, Nk, cols)];
            const int x = (int)(line / cols);
            const int j3 = x % g3, j2 = (x / g3) % g2, j1 = x / (g2 * g3);
            const int i3 = kk % n3, i2 = (kk / n3) % n2, i1 = kk / (n2 * n3);
            double2 p1 = ph[po1 + i1 * g1 + j1], p2 = ph[po2 + i2 * g2 + j2], p3 = ph[po3 + i3 * g3 + j3];
            double2 p12 = cmul(p1, p2);
            double2 p = cmul(p12, p3);
            C2 pc;
            pc.x = (T)p.x;
            pc.y = (T)p.y;
            v = cmul(v, pc);
        }
        buf[e] = v;
    }
    __syncthreads();
    dft3<T, NMAX>(buf, tw_lds, n1, n2, n3, L, false);

    // line 4: multiply by W(x, R)
    for (int e = threadIdx.x; e < Nk * L; e += blockDim.x) {
        const int r = e / L, l = e - r * L;
        const long long line = line0 + l;
        if (line < total) {
            const int x = (int)(line / cols);
            const int r23 = r % (n2 * n3), r1 = r / (n2 * n3);
            const T w = W[(size_t)x * Nk + (size_t)r23 * n1 + r1];
            C2 v = buf[e];
            v.x *= w;
            v.y *= w;
            buf[e] = v;
        }
    }
    __syncthreads();
    dft3<T, NMAX>(buf, tw_lds, n1, n2, n3, L, true);

    // store, with the e^{-ik.x} phase of line 6 and the 1/Nk of the unitary pair
    for (int e = threadIdx.x; e < Nk * L; e += blockDim.x) {
        const int kk = e / L, l = e - kk * L;
        const long long line = line0 + l;
        if (line < total) {
            const int x = (int)(line / cols);
            const int j3 = x % g3, j2 = (x / g3) % g2, j1 = x / (g2 * g3);
            const int i3 = kk % n3, i2 = (kk / n3) % n2, i1 = kk / (n2 * n3);
            double2 p1 = ph[po1 + i1 * g1 + j1], p2 = ph[po2 + i2 * g2 + j2], p3 = ph[po3 + i3 * g3 + j3];
            double2 p = cmul(cmul(p1, p2), p3);
            C2 pc;
            pc.x = (T)p.x * inv_nk;
            pc.y = -(T)p.y * inv_nk;
            phi[phi_index(line, kk, Nk, cols)] = cmul(buf[e], pc);
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Power-of-two k grids (every axis 1, 2, 4, 8 or 16): radix-2 FFTs in registers.
// Five phases, three of them through LDS:
//   P1 load z-pencils from HBM, phase e^{+ik.x}, forward FFT along k3  -> LDS
//   P2 forward FFT along k2                                            (LDS -> LDS)
//   P3 forward FFT along k1, multiply by W(x, R), inverse FFT along k1  (LDS -> LDS)
//   P4 inverse FFT along k2                                            (LDS -> LDS)
//   P5 inverse FFT along k3, phase e^{-ik.x} / Nk, store z-pencils to HBM
// Threads map to pencils with the line index fastest, so 16 consecutive lanes
// touch 16 consecutive lines (contiguous in HBM and conflict-free in LDS).

// e^{2 pi i q / 16}, q = 0..15 (cos and sin of multiples of pi/8)
__device__ __forceinline__ void unit16(int q, double& c, double& s) {
    constexpr double c1 = 0.92387953251128674, c2 = 0.70710678118654752, c3 = 0.38268343236508977;
    const double cq[8] = {1.0, c1, c2, c3, 0.0, -c3, -c2, -c1};  // cos(q pi / 8), q < 8
    const double sq[8] = {0.0, c3, c2, c1, 1.0, c1, c2, c3};     // sin(q pi / 8), q < 8
    q &= 15;
    const double sgn = q < 8 ? 1.0 : -1.0;
    c = sgn * cq[q & 7];
    s = sgn * sq[q & 7];
}

// In-place radix-2 DIT transform X[a] = sum_b x[b] e^{sgn 2 pi i a b / N}, N a power of two <= 16.
template <typename T, int N, int NMAX>
__device__ __forceinline__ void fft_reg(typename C2T<T>::t (&v)[NMAX], bool inverse) {
    typedef typename C2T<T>::t C2;
    if (N == 1) return;
    constexpr int LOG = N == 2 ? 1 : N == 4 ? 2 : N == 8 ? 3 : 4;
    // bit reversal
#pragma unroll
    for (int i = 0; i < N; ++i) {
        int r = 0;
#pragma unroll
        for (int b = 0; b < LOG; ++b) r |= ((i >> b) & 1) << (LOG - 1 - b);
        if (r > i) {
            C2 t = v[i];
            v[i] = v[r];
            v[r] = t;
        }
    }
#pragma unroll
    for (int m = 2; m <= N; m *= 2) {
#pragma unroll
        for (int j = 0; j < m / 2; ++j) {
            double c, sn;
            unit16(j * (16 / m), c, sn);
            const T wr = (T)c, wi = (T)(inverse ? -sn : sn);
#pragma unroll
            for (int k0 = 0; k0 < N; k0 += m) {
                C2 u = v[k0 + j], t = v[k0 + j + m / 2];
                C2 tw;
                tw.x = t.x * wr - t.y * wi;
                tw.y = t.x * wi + t.y * wr;
                v[k0 + j].x = u.x + tw.x;
                v[k0 + j].y = u.y + tw.y;
                v[k0 + j + m / 2].x = u.x - tw.x;
                v[k0 + j + m / 2].y = u.y - tw.y;
            }
        }
    }
}

template <typename T, int NMAX>
__device__ __forceinline__ void fft_any(typename C2T<T>::t (&v)[NMAX], int n, bool inverse) {
    if (NMAX >= 2 && n == 2) fft_reg<T, (NMAX >= 2 ? 2 : 1), NMAX>(v, inverse);
    if (NMAX >= 4 && n == 4) fft_reg<T, (NMAX >= 4 ? 4 : 1), NMAX>(v, inverse);
    if (NMAX >= 8 && n == 8) fft_reg<T, (NMAX >= 8 ? 8 : 1), NMAX>(v, inverse);
    if (NMAX >= 16 && n == 16) fft_reg<T, (NMAX >= 16 ? 16 : 1), NMAX>(v, inverse);
}

__device__ __forceinline__ double2 phase_of(const double2* __restrict__ ph, int kk, int x, int n2, int n3,
                                            int g1, int g2, int g3, int po1, int po2, int po3) {
    const int j3 = x % g3, j2 = (x / g3) % g2, j1 = x / (g2 * g3);
    const int i3 = kk % n3, i2 = (kk / n3) % n2, i1 = kk / (n2 * n3);
    const double2 p1 = ph[po1 + i1 * g1 + j1], p2 = ph[po2 + i2 * g2 + j2], p3 = ph[po3 + i3 * g3 + j3];
    return cmul(cmul(p1, p2), p3);
}

// One LDS pass along an axis of extent n and k-stride st (P2 and P4).
template <typename T, int NMAX>
__device__ __forceinline__ void lds_pass(typename C2T<T>::t* buf, int n, int st, int Nk, int L,
                                         bool inverse) {
    typedef typename C2T<T>::t C2;
    const int npen = (Nk / n) * L;
    for (int p = threadIdx.x; p < npen; p += blockDim.x) {
        const int l = p % L, u = p / L;
        const int base = (u / st) * (n * st) + (u % st);
        C2 v[NMAX];
#pragma unroll
        for (int b = 0; b < NMAX; ++b) v[b] = buf[(base + (b < n ? b : 0) * st) * L + l];
        fft_any<T, NMAX>(v, n, inverse);
#pragma unroll
        for (int b = 0; b < NMAX; ++b)
            if (b < n) buf[(base + b * st) * L + l] = v[b];
    }
}

template <typename T, int NMAX>
__global__ __launch_bounds__(256) void fft_w_pow2_kernel(
    typename C2T<T>::t* __restrict__ phi, const T* __restrict__ W, const double2* __restrict__ ph,
    int n1, int n2, int n3, int g1, int g2, int g3, int po1, int po2, int po3, int Nx, int cols,
    int L) {
    typedef typename C2T<T>::t C2;
    extern __shared__ __align__(16) unsigned char smem[];
    C2* buf = reinterpret_cast<C2*>(smem);  // [Nk][L]
    const int Nk = n1 * n2 * n3;
    const int s3 = __ffs(n3) - 1, s2 = __ffs(n2) - 1;   // log2 of the power-of-two extents
    const long long total = (long long)Nx * cols;
    const long long line0 = (long long)blockIdx.x * L;
    // the block's L lines lie in one x-block: element (kk, l) is at kbase + kk * xbc + l
    const long long xbc = (long long)kXB * cols;
    const long long xblk = line0 / xbc;
    const size_t kbase = (size_t)(xblk * Nk) * xbc + (size_t)(line0 - xblk * xbc);
    // every pencil loop below strides by 256 = a multiple of L, so a thread keeps one line
    const int l = threadIdx.x % L;
    const long long line = line0 + l;
    const bool ok = line < total;
    const int x = ok ? (int)(line / cols) : 0;
    const int j3 = x % g3, j2 = (x / g3) % g2, j1 = x / (g2 * g3);
    const double2* ph1 = ph + po1 + j1;
    const double2* ph2 = ph + po2 + j2;
    const T* wrow = W + (size_t)x * Nk;
    C2* pl = phi + kbase + l;
    // e^{ik.x} = p1(i1) p2(i2) p3(i3): the k3 factors are the same for every pencil of this
    // thread's line, the (k1, k2) factor is one product per pencil
    C2 q3[NMAX];
#pragma unroll
    for (int b = 0; b < NMAX; ++b) {
        const double2 t = ph[po3 + (b < n3 ? b : 0) * g3 + j3];
        q3[b].x = (T)t.x;
        q3[b].y = (T)t.y;
    }
    auto pencil_phase = [&](int u) {
        const double2 a = cmul(ph1[(u >> s2) * g1], ph2[(u & (n2 - 1)) * g2]);
        C2 r;
        r.x = (T)a.x;
        r.y = (T)a.y;
        return r;
    };

    // P1: HBM -> registers, phase, FFT along k3 -> LDS.  Addresses are clamped instead of
    // branched on, so all loads of a pencil are in flight together (padding rows of the
    // x-block are inside the allocation; their values are masked to zero).
    {
        const int npen = (Nk >> s3) * L;
        for (int p = threadIdx.x; p < npen; p += blockDim.x) {
            const int u = p / L;
            C2 v[NMAX];
#pragma unroll
            for (int b = 0; b < NMAX; ++b) {
                const int bb = b < n3 ? b : 0;
                v[b] = pl[(size_t)((u << s3) + bb) * xbc];
            }
            const C2 a = pencil_phase(u);
#pragma unroll
            for (int b = 0; b < NMAX; ++b) {
                C2 pc = cmul(a, q3[b]);
                pc.x = ok ? pc.x : (T)0;
                pc.y = ok ? pc.y : (T)0;
                v[b] = cmul(v[b], pc);
            }
            fft_any<T, NMAX>(v, n3, false);
#pragma unroll
            for (int b = 0; b < NMAX; ++b)
                if (b < n3) buf[((u << s3) + b) * L + l] = v[b];
        }
    }
    __syncthreads();
    // P2
    if (n2 > 1) {
        lds_pass<T, NMAX>(buf, n2, n3, Nk, L, false);
        __syncthreads();
    }
    // P3: FFT along k1, W(x, R), inverse FFT along k1
    {
        const int st = n2 * n3;
        const int npen = st * L;
        for (int p = threadIdx.x; p < npen; p += blockDim.x) {
            const int u = p / L;  // R index within (k2, k3)
            C2 v[NMAX];
#pragma unroll
            for (int b = 0; b < NMAX; ++b) v[b] = buf[(u + (b < n1 ? b : 0) * st) * L + l];
            fft_any<T, NMAX>(v, n1, false);
            // W is stored [x][R2 R3][R1]: the n1 values of this pencil are contiguous
            T wv[NMAX];
            if (n1 == NMAX) {
                const WVec<T, NMAX> wl = reinterpret_cast<const WVec<T, NMAX>*>(wrow)[u];
#pragma unroll
                for (int b = 0; b < NMAX; ++b) wv[b] = wl.v[b];
            } else {
#pragma unroll
                for (int b = 0; b < NMAX; ++b) wv[b] = wrow[u * n1 + (b < n1 ? b : 0)];
            }
#pragma unroll
            for (int b = 0; b < NMAX; ++b) {
                const T w = ok ? wv[b] : (T)0;
                v[b].x *= w;
                v[b].y *= w;
            }
            fft_any<T, NMAX>(v, n1, true);
#pragma unroll
            for (int b = 0; b < NMAX; ++b)
                if (b < n1) buf[(u + b * st) * L + l] = v[b];
        }
    }
    __syncthreads();
    // P4
    if (n2 > 1) {
        lds_pass<T, NMAX>(buf, n2, n3, Nk, L, true);
        __syncthreads();
    }
    // P5: inverse FFT along k3, phase e^{-ik.x} / Nk, registers -> HBM
    if (ok) {
        const T inv_nk = (T)(1.0 / (double)Nk);
        const int npen = (Nk >> s3) * L;
        for (int p = threadIdx.x; p < npen; p += blockDim.x) {
            const int u = p / L;
            C2 v[NMAX];
#pragma unroll
            for (int b = 0; b < NMAX; ++b) v[b] = buf[((u << s3) + (b < n3 ? b : 0)) * L + l];
            fft_any<T, NMAX>(v, n3, true);
            const C2 a = pencil_phase(u);
            C2 o[NMAX];
#pragma unroll
            for (int b = 0; b < NMAX; ++b) {
                C2 pc = cmul(a, q3[b]);
                pc.x = pc.x * inv_nk;
                pc.y = -pc.y * inv_nk;
                o[b] = cmul(v[b], pc);
            }
#pragma unroll
            for (int b = 0; b < NMAX; ++b)
                if (b < n3) pl[(size_t)((u << s3) + b) * xbc] = o[b];
        }
    }
}

bool is_pow2_grid(const ocean_bse_s* h) {
    for (int a = 0; a < 3; ++a) {
        const int n = h->nk[a];
        if (n != 1 && n != 2 && n != 4 && n != 8 && n != 16) return false;
    }
    return true;
}

template <typename T>
hipError_t fft_dispatch(ocean_bse_s* h, int cols, const T* W) {
    typedef typename C2T<T>::t C2;
    // lines of one block must stay inside one x-block of the phi layout
    int L = h->fft_lines;
    while (L > 1 && ((long long)kXB * cols) % L != 0) L /= 2;
    const long long total = (long long)h->Nx * cols;
    const unsigned nblk = (unsigned)((total + L - 1) / L);
    const size_t lds = sizeof(C2) * (3 * kMaxDft + (size_t)h->Nk * L);
    const int nmax = std::max(h->nk[0], std::max(h->nk[1], h->nk[2]));
    C2* phi = static_cast<C2*>(h->ws.phi);
    const double2* ph = reinterpret_cast<const double2*>(h->phase);
    const double2* tw = reinterpret_cast<const double2*>(h->twiddle);
    if (is_pow2_grid(h)) {
        const size_t lds2 = sizeof(C2) * (size_t)h->Nk * L;
#define OCEAN_POW2_ARGS                                                                            \
    phi, W, ph, h->nk[0], h->nk[1], h->nk[2], h->nx[0], h->nx[1], h->nx[2], h->phase_off[0],        \
        h->phase_off[1], h->phase_off[2], h->Nx, cols, L
        if (nmax <= 2)
            fft_w_pow2_kernel<T, 2><<<nblk, 256, lds2, h->stream>>>(OCEAN_POW2_ARGS);
        else if (nmax <= 4)
            fft_w_pow2_kernel<T, 4><<<nblk, 256, lds2, h->stream>>>(OCEAN_POW2_ARGS);
        else if (nmax <= 8)
            fft_w_pow2_kernel<T, 8><<<nblk, 256, lds2, h->stream>>>(OCEAN_POW2_ARGS);
        else
            fft_w_pow2_kernel<T, 16><<<nblk, 256, lds2, h->stream>>>(OCEAN_POW2_ARGS);
#undef OCEAN_POW2_ARGS
        return hipGetLastError();
    }
#define OCEAN_FFT_ARGS                                                                          \
    phi, W, ph, tw, h->nk[0], h->nk[1], h->nk[2], h->nx[0], h->nx[1], h->nx[2], h->phase_off[0], \
        h->phase_off[1], h->phase_off[2], h->tw_off[0], h->tw_off[1], h->tw_off[2], h->Nx, cols, L
    if (nmax <= 2)
        fft_w_kernel<T, 2><<<nblk, 256, lds, h->stream>>>(OCEAN_FFT_ARGS);
    else if (nmax <= 4)
        fft_w_kernel<T, 4><<<nblk, 256, lds, h->stream>>>(OCEAN_FFT_ARGS);
    else if (nmax <= 8)
        fft_w_kernel<T, 8><<<nblk, 256, lds, h->stream>>>(OCEAN_FFT_ARGS);
    else
        fft_w_kernel<T, 16><<<nblk, 256, lds, h->stream>>>(OCEAN_FFT_ARGS);
#undef OCEAN_FFT_ARGS
    return hipGetLastError();
}

}  // namespace

size_t fft_lds_bytes(const ocean_bse_s* h, int lines) {
    const size_t elem = h->precision == OCEAN_PREC_FP64 ? 16 : 8;
    return elem * (3 * kMaxDft + (size_t)h->Nk * lines);
}

hipError_t launch_fft_w(ocean_bse_s* h, int cols) {
    const int slot = prof_begin(h, "fft_w");
    hipError_t e;
    if (h->precision == OCEAN_PREC_FP64)
        e = fft_dispatch<double>(h, cols, h->W64);
    else
        e = fft_dispatch<float>(h, cols, h->W32);
    prof_end(h, slot);
    return e;
}

}  // namespace ocean
