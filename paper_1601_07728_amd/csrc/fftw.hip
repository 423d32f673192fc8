// k-grid transform and screened-potential multiply of Algorithm 1 (section 3.2.1):
//
//   phi(x, R)  = Nk^{-1/2} sum_k e^{+ik.R} phi(x, k)      (k -> R)
//   phi(x, R) *= W(x, R)                                  (screened potential, diagonal in x)
//   phi'(x, k) = Nk^{-1/2} sum_R e^{-ik.R} phi(x, R)       (R -> k)
//
// The Bloch phase e^{+-ik.x} of the band projections is normally carried by the stored u;
// for a borrowed FP64 u the kernels apply it here on the way in and out.  The product of
// the two Nk^{-1/2} is folded into the W table.
//
// A line is one (x, column) pair; its Nk values sit in the x-blocked phi layout.  A block
// stages L lines in LDS as [k][line], runs the separable small DFTs along the three k axes,
// multiplies by W and transforms back, then writes the lines in place.  The pass is
// HBM-bound: phi is read once and written once.
#include <type_traits>

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

template <typename T, typename S, int NMAX>
__global__ __launch_bounds__(256) void fft_w_kernel(
    S* __restrict__ phi, const T* __restrict__ W, const double2* __restrict__ ph,
    const double2* __restrict__ tw, int n1, int n2, int n3, int g1, int g2, int g3, int po1,
    int po2, int po3, int to1, int to2, int to3, int Nx, int cols, int L, int phase) {
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
    // load, with the e^{+ik.x} phase unless u carries it
    for (int e = threadIdx.x; e < Nk * L; e += blockDim.x) {
        const int kk = e / L, l = e - kk * L;
        const long long line = line0 + l;
        C2 v;
        v.x = 0;
        v.y = 0;
        if (line < total) {
            v = phi_load<C2>(&phi[phi_index(line, kk, Nk, cols)]);
        }
        if (line < total && phase) {
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

    // screened potential: multiply by W(x, R)
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

    // store, with the e^{-ik.x} phase unless u carries it (the 1/Nk of the
    // unitary pair is in W)
    for (int e = threadIdx.x; e < Nk * L; e += blockDim.x) {
        const int kk = e / L, l = e - kk * L;
        const long long line = line0 + l;
        if (line < total && !phase) phi_store(&phi[phi_index(line, kk, Nk, cols)], buf[e]);
        if (line < total && phase) {
            const int x = (int)(line / cols);
            const int j3 = x % g3, j2 = (x / g3) % g2, j1 = x / (g2 * g3);
            const int i3 = kk % n3, i2 = (kk / n3) % n2, i1 = kk / (n2 * n3);
            double2 p1 = ph[po1 + i1 * g1 + j1], p2 = ph[po2 + i2 * g2 + j2], p3 = ph[po3 + i3 * g3 + j3];
            double2 p = cmul(cmul(p1, p2), p3);
            C2 pc;
            pc.x = (T)p.x;
            pc.y = -(T)p.y;
            phi_store(&phi[phi_index(line, kk, Nk, cols)], cmul(buf[e], pc));
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

// t * e^{sgn 2 pi i q / 16} (sgn = -1 for the inverse).  q is a constant once the radix-2
// loops are unrolled, so the multiples of pi/4 reduce to swaps, negations and one scale.
template <typename T, bool INV>
__device__ __forceinline__ typename C2T<T>::t twiddle16(typename C2T<T>::t t, int q) {
    typedef typename C2T<T>::t C2;
    const T s = INV ? (T)-1 : (T)1;
    const T r = (T)0.70710678118654752440;
    C2 o;
    switch (q & 15) {
        case 0: return t;
        case 4: o.x = -s * t.y; o.y = s * t.x; return o;
        case 8: o.x = -t.x; o.y = -t.y; return o;
        case 12: o.x = s * t.y; o.y = -s * t.x; return o;
        case 2: o.x = r * (t.x - s * t.y); o.y = r * (t.y + s * t.x); return o;
        case 6: o.x = r * (-t.x - s * t.y); o.y = r * (s * t.x - t.y); return o;
        case 10: o.x = r * (s * t.y - t.x); o.y = r * (-t.y - s * t.x); return o;
        case 14: o.x = r * (t.x + s * t.y); o.y = r * (t.y - s * t.x); return o;
        default: {
            double c, sn;
            unit16(q, c, sn);
            const T wr = (T)c, wi = s * (T)sn;
            o.x = t.x * wr - t.y * wi;
            o.y = t.x * wi + t.y * wr;
            return o;
        }
    }
}

// In-place radix-2 DIT transform X[a] = sum_b x[b] e^{sgn 2 pi i a b / N}, N a power of two <= 16.
template <typename T, int N, int NMAX, bool INV>
__device__ __forceinline__ void fft_reg(typename C2T<T>::t (&v)[NMAX]) {
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
#pragma unroll
            for (int k0 = 0; k0 < N; k0 += m) {
                const C2 u = v[k0 + j];
                const C2 tw = twiddle16<T, INV>(v[k0 + j + m / 2], j * (16 / m));
                v[k0 + j].x = u.x + tw.x;
                v[k0 + j].y = u.y + tw.y;
                v[k0 + j + m / 2].x = u.x - tw.x;
                v[k0 + j + m / 2].y = u.y - tw.y;
            }
        }
    }
}

template <typename T, int NMAX, bool INV>
__device__ __forceinline__ void fft_any(typename C2T<T>::t (&v)[NMAX], int n) {
    if (NMAX >= 2 && n == 2) fft_reg<T, (NMAX >= 2 ? 2 : 1), NMAX, INV>(v);
    if (NMAX >= 4 && n == 4) fft_reg<T, (NMAX >= 4 ? 4 : 1), NMAX, INV>(v);
    if (NMAX >= 8 && n == 8) fft_reg<T, (NMAX >= 8 ? 8 : 1), NMAX, INV>(v);
    if (NMAX >= 16 && n == 16) fft_reg<T, (NMAX >= 16 ? 16 : 1), NMAX, INV>(v);
}

// LDS layout of the power-of-two kernel: element (k, l) at k L + l + (k >> s3) pad.  The
// padding after every run of n3 k rows is chosen so that consecutive k3 pencils (the lanes
// of one P1/P5 access) fall into consecutive banks.
inline int pow2_pad(int elem_bytes, int n3, int L) {
    const int M = 256 / elem_bytes;  // elements in one sweep of the 64 four-byte banks
    return (M - ((n3 - 1) * L) % M) % M;
}

// One LDS pass of the k2 axis (P2 forward, P4 inverse).
template <typename T, int NMAX, bool INV>
__device__ __forceinline__ void lds_pass_k2(typename C2T<T>::t* buf, int s1, int s2, int s3, int lL, int l,
                                            int pad) {
    typedef typename C2T<T>::t C2;
    const int n2 = 1 << s2, n3 = 1 << s3;
    const int npen = (1 << (s1 + s3)) << lL;
    for (int p = threadIdx.x; p < npen; p += blockDim.x) {
        const int u = p >> lL;  // (i1, i3)
        const int base = ((u >> s3) << (s2 + s3)) + (u & (n3 - 1));
        C2 v[NMAX];
#pragma unroll
        for (int b = 0; b < NMAX; ++b) {
            const int k = base + ((b < n2 ? b : 0) << s3);
            v[b] = buf[(k << lL) + l + (k >> s3) * pad];
        }
        fft_any<T, NMAX, INV>(v, n2);
#pragma unroll
        for (int b = 0; b < NMAX; ++b) {
            const int k = base + (b << s3);
            if (b < n2) buf[(k << lL) + l + (k >> s3) * pad] = v[b];
        }
    }
}

template <typename T, typename S, int NMAX>
__global__ __launch_bounds__(256) void fft_w_pow2_kernel(
    S* __restrict__ phi, const T* __restrict__ W, const double2* __restrict__ ph,
    int s1, int s2, int s3, int g1, int g2, int g3, int po1, int po2, int po3, int total, int cols,
    int lL, int pad, int phase) {
    typedef typename C2T<T>::t C2;
    extern __shared__ __align__(16) unsigned char smem[];
    C2* buf = reinterpret_cast<C2*>(smem);
    const int n1 = 1 << s1, n2 = 1 << s2, n3 = 1 << s3;
    const int sk = s1 + s2 + s3;
    const int Nk = 1 << sk;
    const int L = 1 << lL;
    // Workgroups are dealt round-robin to the 8 XCDs; renumber them so that each XCD takes a
    // contiguous run of line groups: neighbouring groups share cache lines of phi when L
    // lines span less than a line, and those now meet in one XCD's L2.
    const unsigned nblk = gridDim.x, q8 = nblk / 8, r8 = nblk % 8;
    const unsigned xcd = blockIdx.x % 8, pos = blockIdx.x / 8;
    const int lblk = (int)(xcd * q8 + (xcd < r8 ? xcd : r8) + pos);
    const int line0 = lblk << lL;
    // the block's L lines lie in one x-block: element (k, l) is at kbase + k xbc + l
    const int xbc = kXB * cols;
    const int xblk = line0 / xbc;
    const size_t kbase = (size_t)xblk * Nk * xbc + (size_t)(line0 - xblk * xbc);
    // every pencil loop strides by 256, a multiple of L, so a thread keeps one line
    const int l = threadIdx.x & (L - 1);
    const int line = line0 + l;
    const bool ok = line < total;
    const int x = ok ? line / cols : 0;
    const int j3 = x % g3, j2 = (x / g3) % g2, j1 = x / (g2 * g3);
    const double2* ph1 = ph + po1 + j1;
    const double2* ph2 = ph + po2 + j2;
    const T* wrow = W + (size_t)x * Nk;
    S* pl = phi + kbase + l;
    auto lidx = [&](int k) { return (k << lL) + l + (k >> s3) * pad; };
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
    const int npen3 = (Nk >> s3) << lL;

    // P1: HBM -> registers, phase, FFT along k3 -> LDS.  Addresses are clamped instead of
    // branched on, so all loads are in flight together (padding rows of the x-block are
    // inside the allocation; their values are masked to zero).  UP pencils per thread are
    // loaded before any of them is transformed.
    {
        constexpr int UP = sizeof(T) == 4 ? 4 : 2;
        for (int p0 = threadIdx.x; p0 < npen3; p0 += UP * blockDim.x) {
            C2 v[UP][NMAX];
#pragma unroll
            for (int q = 0; q < UP; ++q) {
                const int p = p0 + q * (int)blockDim.x;
                const int u = (p < npen3 ? p : p0) >> lL;
#pragma unroll
                for (int b = 0; b < NMAX; ++b) v[q][b] = phi_load<C2>(&pl[((u << s3) + (b < n3 ? b : 0)) * xbc]);
            }
#pragma unroll
            for (int q = 0; q < UP; ++q) {
                const int p = p0 + q * (int)blockDim.x;
                if (p >= npen3) break;
                const int u = p >> lL;
                if (phase) {
                    const C2 a = pencil_phase(u);
#pragma unroll
                    for (int b = 0; b < NMAX; ++b) {
                        C2 pc = cmul(a, q3[b]);
                        pc.x = ok ? pc.x : (T)0;
                        pc.y = ok ? pc.y : (T)0;
                        v[q][b] = cmul(v[q][b], pc);
                    }
                } else if (!ok) {
#pragma unroll
                    for (int b = 0; b < NMAX; ++b) v[q][b].x = v[q][b].y = (T)0;
                }
                fft_any<T, NMAX, false>(v[q], n3);
#pragma unroll
                for (int b = 0; b < NMAX; ++b)
                    if (b < n3) buf[lidx((u << s3) + b)] = v[q][b];
            }
        }
    }
    __syncthreads();
    if (n2 > 1) {  // P2
        lds_pass_k2<T, NMAX, false>(buf, s1, s2, s3, lL, l, pad);
        __syncthreads();
    }
    // P3: FFT along k1, W(x, R), inverse FFT along k1
    {
        const int s23 = s2 + s3;
        const int npen = (1 << s23) << lL;
        for (int p = threadIdx.x; p < npen; p += blockDim.x) {
            const int u = p >> lL;  // R index within (k2, k3)
            C2 v[NMAX];
#pragma unroll
            for (int b = 0; b < NMAX; ++b) v[b] = buf[lidx(u + ((b < n1 ? b : 0) << s23))];
            fft_any<T, NMAX, false>(v, n1);
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
            fft_any<T, NMAX, true>(v, n1);
#pragma unroll
            for (int b = 0; b < NMAX; ++b)
                if (b < n1) buf[lidx(u + (b << s23))] = v[b];
        }
    }
    __syncthreads();
    if (n2 > 1) {  // P4
        lds_pass_k2<T, NMAX, true>(buf, s1, s2, s3, lL, l, pad);
        __syncthreads();
    }
    // P5: inverse FFT along k3, phase e^{-ik.x} (unless u carries it), registers -> HBM
    if (ok) {
        for (int p = threadIdx.x; p < npen3; p += blockDim.x) {
            const int u = p >> lL;
            C2 v[NMAX];
#pragma unroll
            for (int b = 0; b < NMAX; ++b) v[b] = buf[lidx((u << s3) + (b < n3 ? b : 0))];
            fft_any<T, NMAX, true>(v, n3);
            if (phase) {
                const C2 a = pencil_phase(u);
#pragma unroll
                for (int b = 0; b < NMAX; ++b) {
                    C2 pc = cmul(a, q3[b]);
                    pc.y = -pc.y;
                    v[b] = cmul(v[b], pc);
                }
            }
#pragma unroll
            for (int b = 0; b < NMAX; ++b)
                if (b < n3) phi_store(&pl[((u << s3) + b) * xbc], v[b]);
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Cubic grids N^3 (N = 4 or 8) with the extent N and the line count L fixed at compile time:
// the pencil loops unroll completely and every LDS address is a per-thread base plus a
// constant, so the five phases are almost pure transform arithmetic.  u normally carries
// the Bloch phase (PH = false); PH = true applies e^{+-ik.x} here for a borrowed FP64 u.
template <typename T, typename S, int N, int L, bool PH>
__global__ __launch_bounds__(256) void fft_w_cube_kernel(
    S* __restrict__ phi, const T* __restrict__ W, const double2* __restrict__ ph,
    int g1, int g2, int g3, int po1, int po2, int po3, int total, int cols) {
    typedef typename C2T<T>::t C2;
    constexpr int NK = N * N * N, NP = N * N;   // k points; pencils of one line along an axis
    constexpr int E = sizeof(C2);
    constexpr int M = 256 / E;                  // elements in one sweep of the 64 LDS banks
    constexpr int PAD = (M - ((N - 1) * L) % M) % M;
    constexpr int TPL = 256 / L;                // pencil stride between a thread's pencils
    constexpr int PPT = (NP * L + 255) / 256;   // pencils per thread and pass
    constexpr int RUN = N * L + PAD;            // LDS stride of one k3 pencil
    extern __shared__ __align__(16) unsigned char smem[];
    C2* buf = reinterpret_cast<C2*>(smem);      // element (k, l) at k L + l + (k / N) PAD

    // XCD-contiguous renumbering of the workgroups (see fft_w_pow2_kernel)
    const unsigned nblk = gridDim.x, q8 = nblk / 8, r8 = nblk % 8;
    const unsigned xcd = blockIdx.x % 8, pos = blockIdx.x / 8;
    const int lblk = (int)(xcd * q8 + (xcd < r8 ? xcd : r8) + pos);
    const int line0 = lblk * L;
    const int xbc = kXB * cols;
    const int xblk = line0 / xbc;
    const size_t kbase = (size_t)xblk * NK * xbc + (size_t)(line0 - xblk * xbc);
    const int l = threadIdx.x % L, u0 = threadIdx.x / L;
    const int line = line0 + l;
    const bool ok = line < total;
    const int x = ok ? line / cols : 0;
    const T* wrow = W + (size_t)x * NK;
    S* pl = phi + kbase + l;

    C2 q3[N];
    const double2* ph1 = ph + po1;
    const double2* ph2 = ph + po2;
    int j1 = 0, j2 = 0;
    if (PH) {
        const int j3 = x % g3;
        j2 = (x / g3) % g2;
        j1 = x / (g2 * g3);
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const double2 t = ph[po3 + b * g3 + j3];
            q3[b].x = (T)t.x;
            q3[b].y = (T)t.y;
        }
    }
    // e^{ik.x} of pencil u = (i1, i2) and point b along k3, or its conjugate
    auto phase_of = [&](int u, int b, bool conj) {
        const double2 a = cmul(ph1[(u / N) * g1 + j1], ph2[(u % N) * g2 + j2]);
        C2 ac;
        ac.x = (T)a.x;
        ac.y = (T)a.y;
        C2 r = cmul(ac, q3[b]);
        if (conj) r.y = -r.y;
        return r;
    };

    // P1: HBM -> registers (all of this thread's pencils first), FFT along k3 -> LDS
    {
        C2 v[PPT][N];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int u = u0 + j * TPL;
            if (u < NP) {
#pragma unroll
                for (int b = 0; b < N; ++b) v[j][b] = phi_load<C2>(&pl[(u * N + b) * xbc]);
            }
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int u = u0 + j * TPL;
            if (u >= NP) continue;
#pragma unroll
            for (int b = 0; b < N; ++b) {
                if (!ok) v[j][b].x = v[j][b].y = (T)0;
                if (PH) v[j][b] = cmul(v[j][b], phase_of(u, b, false));
            }
            fft_reg<T, N, N, false>(v[j]);
#pragma unroll
            for (int b = 0; b < N; ++b) buf[u * RUN + l + b * L] = v[j][b];
        }
    }
    __syncthreads();
    // P2 / P4: the k2 axis; pencil u = (i1, i3)
    auto k2_pass = [&](auto inv) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int u = u0 + j * TPL;
            if (u >= NP) continue;
            const int base = ((u / N) * NP + (u % N)) * L + l + (u / N) * N * PAD;
            C2 v[N];
#pragma unroll
            for (int b = 0; b < N; ++b) v[b] = buf[base + b * (N * L + PAD)];
            fft_reg<T, N, N, decltype(inv)::value>(v);
#pragma unroll
            for (int b = 0; b < N; ++b) buf[base + b * (N * L + PAD)] = v[b];
        }
    };
    k2_pass(std::false_type{});
    __syncthreads();
    // P3: FFT along k1, W(x, R) (stored [x][R2 R3][R1], 1/Nk included), inverse FFT along k1
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int u = u0 + j * TPL;  // (i2, i3)
        if (u >= NP) continue;
        const int base = u * L + l + (u / N) * PAD;
        constexpr int STEP = NP * L + N * PAD;
        C2 v[N];
#pragma unroll
        for (int b = 0; b < N; ++b) v[b] = buf[base + b * STEP];
        fft_reg<T, N, N, false>(v);
        const WVec<T, N> wl = reinterpret_cast<const WVec<T, N>*>(wrow)[u];
#pragma unroll
        for (int b = 0; b < N; ++b) {
            v[b].x *= wl.v[b];
            v[b].y *= wl.v[b];
        }
        fft_reg<T, N, N, true>(v);
#pragma unroll
        for (int b = 0; b < N; ++b) buf[base + b * STEP] = v[b];
    }
    __syncthreads();
    k2_pass(std::true_type{});
    __syncthreads();
    // P5: inverse FFT along k3 -> HBM
    if (ok) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int u = u0 + j * TPL;
            if (u >= NP) continue;
            C2 v[N];
#pragma unroll
            for (int b = 0; b < N; ++b) v[b] = buf[u * RUN + l + b * L];
            fft_reg<T, N, N, true>(v);
#pragma unroll
            for (int b = 0; b < N; ++b) {
                if (PH) v[b] = cmul(v[b], phase_of(u, b, true));
                phi_store(&pl[(u * N + b) * xbc], v[b]);
            }
        }
    }
}

// Two adjacent stored phi values (lines l, l + 1 of one k row) moved as one access: 8 bytes
// for bf16 pairs, 16 for FP32 pairs.
template <typename S> struct PairW;
template <> struct PairW<bf16c> { typedef uint2 t; };
template <> struct PairW<float2> { typedef float4 t; };
__device__ __forceinline__ void pair_unpack(uint2 w, float2& a, float2& b) {
    a = phi_load<float2, bf16c>(reinterpret_cast<const bf16c*>(&w.x));
    b = phi_load<float2, bf16c>(reinterpret_cast<const bf16c*>(&w.y));
}
__device__ __forceinline__ void pair_unpack(float4 w, float2& a, float2& b) {
    a = make_float2(w.x, w.y);
    b = make_float2(w.z, w.w);
}
__device__ __forceinline__ void pair_pack(float2 a, float2 b, uint2& w) {
    phi_store<float2, bf16c>(reinterpret_cast<bf16c*>(&w.x), a);
    phi_store<float2, bf16c>(reinterpret_cast<bf16c*>(&w.y), b);
}
__device__ __forceinline__ void pair_pack(float2 a, float2 b, float4& w) { w = make_float4(a.x, a.y, b.x, b.y); }

// The cube kernel with two lines per thread (FP32 arithmetic, u carrying the Bloch phase,
// N = 8, L >= 8): the same five phases and LDS layout, with every HBM and LDS access moving
// the values of lines l and l + 1 together, so the block issues half as many memory
// instructions for the same bytes.  Lines past `total` (the padding of the last x-block,
// inside the allocation) are transformed as zeros and written back as zeros.
template <typename S, int N, int L>
__global__ __launch_bounds__(256) void fft_w_cube2_kernel(S* __restrict__ phi, const float* __restrict__ W,
                                                          int total, int cols) {
    typedef float2 C2;
    typedef typename PairW<S>::t PW;
    constexpr int NK = N * N * N, NP = N * N;
    constexpr int M = 256 / (int)sizeof(C2);
    constexpr int PAD = (M - ((N - 1) * L) % M) % M;
    constexpr int LP = L / 2;                   // line pairs per block
    constexpr int TPL = 256 / LP;               // pencil stride between a thread's pencils
    constexpr int PPT = NP * LP / 256;          // pencils per thread and pass
    constexpr int RUN = N * L + PAD;
    static_assert(NP * LP % 256 == 0 && PAD % 2 == 0 && L % 2 == 0, "whole pencils, aligned pairs");
    extern __shared__ __align__(16) unsigned char smem[];
    C2* buf = reinterpret_cast<C2*>(smem);      // element (k, l) at k L + l + (k / N) PAD

    // XCD-contiguous renumbering of the workgroups (see fft_w_pow2_kernel)
    const unsigned nblk = gridDim.x, q8 = nblk / 8, r8 = nblk % 8;
    const unsigned xcd = blockIdx.x % 8, pos = blockIdx.x / 8;
    const int lblk = (int)(xcd * q8 + (xcd < r8 ? xcd : r8) + pos);
    const int line0 = lblk * L;
    const int xbc = kXB * cols;
    const int xblk = line0 / xbc;
    const size_t kbase = (size_t)xblk * NK * xbc + (size_t)(line0 - xblk * xbc);
    const int l = 2 * (threadIdx.x % LP), u0 = threadIdx.x / LP;
    const bool ok0 = line0 + l < total, ok1 = line0 + l + 1 < total;
    const float* w0 = W + (size_t)(ok0 ? (line0 + l) / cols : 0) * NK;
    const float* w1 = W + (size_t)(ok1 ? (line0 + l + 1) / cols : 0) * NK;
    S* pl = phi + kbase + l;
    auto lds_get = [&](int e, C2& a, C2& b) {
        const float4 q = *reinterpret_cast<const float4*>(&buf[e]);
        a = make_float2(q.x, q.y);
        b = make_float2(q.z, q.w);
    };
    auto lds_put = [&](int e, C2 a, C2 b) { *reinterpret_cast<float4*>(&buf[e]) = make_float4(a.x, a.y, b.x, b.y); };

    // P1: HBM -> registers, FFT along k3 -> LDS
    {
        PW r[PPT][N];
#pragma unroll
        for (int j = 0; j < PPT; ++j)
#pragma unroll
            for (int b = 0; b < N; ++b) r[j][b] = *reinterpret_cast<const PW*>(&pl[((u0 + j * TPL) * N + b) * xbc]);
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int u = u0 + j * TPL;
            C2 va[N], vb[N];
#pragma unroll
            for (int b = 0; b < N; ++b) {
                pair_unpack(r[j][b], va[b], vb[b]);
                if (!ok0) va[b].x = va[b].y = 0.f;
                if (!ok1) vb[b].x = vb[b].y = 0.f;
            }
            fft_reg<float, N, N, false>(va);
            fft_reg<float, N, N, false>(vb);
#pragma unroll
            for (int b = 0; b < N; ++b) lds_put(u * RUN + l + b * L, va[b], vb[b]);
        }
    }
    __syncthreads();
    auto k2_pass = [&](auto inv) {
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int u = u0 + j * TPL;
            const int base = ((u / N) * NP + (u % N)) * L + l + (u / N) * N * PAD;
            C2 va[N], vb[N];
#pragma unroll
            for (int b = 0; b < N; ++b) lds_get(base + b * (N * L + PAD), va[b], vb[b]);
            fft_reg<float, N, N, decltype(inv)::value>(va);
            fft_reg<float, N, N, decltype(inv)::value>(vb);
#pragma unroll
            for (int b = 0; b < N; ++b) lds_put(base + b * (N * L + PAD), va[b], vb[b]);
        }
    };
    k2_pass(std::false_type{});
    __syncthreads();
    // P3: FFT along k1, W(x, R) of each line's point (stored [x][R2 R3][R1], 1/Nk included),
    // inverse FFT along k1
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int u = u0 + j * TPL;
        const int base = u * L + l + (u / N) * PAD;
        constexpr int STEP = NP * L + N * PAD;
        C2 va[N], vb[N];
#pragma unroll
        for (int b = 0; b < N; ++b) lds_get(base + b * STEP, va[b], vb[b]);
        fft_reg<float, N, N, false>(va);
        fft_reg<float, N, N, false>(vb);
        const WVec<float, N> wa = reinterpret_cast<const WVec<float, N>*>(w0)[u];
        const WVec<float, N> wb = reinterpret_cast<const WVec<float, N>*>(w1)[u];
#pragma unroll
        for (int b = 0; b < N; ++b) {
            const float fa = ok0 ? wa.v[b] : 0.f, fb = ok1 ? wb.v[b] : 0.f;
            va[b].x *= fa;
            va[b].y *= fa;
            vb[b].x *= fb;
            vb[b].y *= fb;
        }
        fft_reg<float, N, N, true>(va);
        fft_reg<float, N, N, true>(vb);
#pragma unroll
        for (int b = 0; b < N; ++b) lds_put(base + b * STEP, va[b], vb[b]);
    }
    __syncthreads();
    k2_pass(std::true_type{});
    __syncthreads();
    // P5: inverse FFT along k3 -> HBM
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int u = u0 + j * TPL;
        C2 va[N], vb[N];
#pragma unroll
        for (int b = 0; b < N; ++b) lds_get(u * RUN + l + b * L, va[b], vb[b]);
        fft_reg<float, N, N, true>(va);
        fft_reg<float, N, N, true>(vb);
#pragma unroll
        for (int b = 0; b < N; ++b) {
            PW w;
            pair_pack(va[b], vb[b], w);
            *reinterpret_cast<PW*>(&pl[(u * N + b) * xbc]) = w;
        }
    }
}

template <typename T, int N, int L>
size_t cube_lds_bytes() {
    typedef typename C2T<T>::t C2;
    constexpr int E = sizeof(C2), M = 256 / E;
    constexpr int PAD = (M - ((N - 1) * L) % M) % M;
    return (size_t)E * ((size_t)N * N * N * L + (size_t)N * N * PAD);
}

template <typename T, typename S, int N, int L>
hipError_t launch_cube(ocean_bse_s* h, S* phi, const T* W, const double2* ph, int total,
                       int cols, bool phase) {
    const unsigned nblk = (unsigned)((total + L - 1) / L);
    const size_t lds = cube_lds_bytes<T, N, L>();
    if constexpr (sizeof(T) == 4 && N == 8 && L >= 8) {
        if (!phase && h->fft_pairs) {
            fft_w_cube2_kernel<S, N, L><<<nblk, 256, lds, h->stream>>>(phi, W, total, cols);
            return hipGetLastError();
        }
    }
#define OCEAN_CUBE_ARGS phi, W, ph, h->nx[0], h->nx[1], h->nx[2], h->phase_off[0], h->phase_off[1], h->phase_off[2], total, cols
    if (phase) {
        if constexpr (sizeof(T) == 8)
            fft_w_cube_kernel<T, S, N, L, true><<<nblk, 256, lds, h->stream>>>(OCEAN_CUBE_ARGS);
        else
            return hipErrorInvalidValue;  // only a borrowed FP64 u is unphased
    } else {
        fft_w_cube_kernel<T, S, N, L, false><<<nblk, 256, lds, h->stream>>>(OCEAN_CUBE_ARGS);
    }
#undef OCEAN_CUBE_ARGS
    return hipGetLastError();
}

// The cube kernel applies when the grid is N^3 with N = 4 or 8 and L is 4, 8 or 16.
bool cube_ok(const ocean_bse_s* h, int L) {
    const int n = h->nk[0];
    return h->nk[1] == n && h->nk[2] == n && (n == 4 || n == 8) && (L == 4 || L == 8 || L == 16);
}

template <typename T, typename S>
hipError_t cube_dispatch(ocean_bse_s* h, S* phi, const T* W, const double2* ph, int total,
                         int cols, int L, bool phase) {
    const int n = h->nk[0];
    if (n == 8) {
        if (L == 4) return launch_cube<T, S, 8, 4>(h, phi, W, ph, total, cols, phase);
        if (L == 8) return launch_cube<T, S, 8, 8>(h, phi, W, ph, total, cols, phase);
        return launch_cube<T, S, 8, 16>(h, phi, W, ph, total, cols, phase);
    }
    if (L == 4) return launch_cube<T, S, 4, 4>(h, phi, W, ph, total, cols, phase);
    if (L == 8) return launch_cube<T, S, 4, 8>(h, phi, W, ph, total, cols, phase);
    return launch_cube<T, S, 4, 16>(h, phi, W, ph, total, cols, phase);
}

bool is_pow2_grid(const ocean_bse_s* h) {
    for (int a = 0; a < 3; ++a) {
        const int n = h->nk[a];
        if (n != 1 && n != 2 && n != 4 && n != 8 && n != 16) return false;
    }
    return true;
}

// T: compute type, S: stored type of phi
template <typename T, typename S>
hipError_t fft_dispatch(ocean_bse_s* h, int cols, const T* W) {
    typedef typename C2T<T>::t C2;
    const int phase = h->u_phased ? 0 : 1;
    // lines of one block must stay inside one x-block of the phi layout
    int L = h->fft_lines;
    while (L > 1 && ((long long)kXB * cols) % L != 0) L /= 2;
    const long long total = (long long)h->Nx * cols;
    const unsigned nblk = (unsigned)((total + L - 1) / L);
    const size_t lds = sizeof(C2) * (3 * kMaxDft + (size_t)h->Nk * L);
    const int nmax = std::max(h->nk[0], std::max(h->nk[1], h->nk[2]));
    S* phi = static_cast<S*>(h->ws.phi);
    const double2* ph = reinterpret_cast<const double2*>(h->phase);
    const double2* tw = reinterpret_cast<const double2*>(h->twiddle);
    if (cube_ok(h, L) && total < (1LL << 31))
        return cube_dispatch<T, S>(h, phi, W, ph, (int)total, cols, L, phase != 0);
    if (is_pow2_grid(h) && total < (1LL << 31)) {
        const int pad = pow2_pad((int)sizeof(C2), h->nk[2], L);
        const size_t lds2 = sizeof(C2) * ((size_t)h->Nk * L + (size_t)(h->Nk / h->nk[2]) * pad);
        int lL = 0;
        while ((1 << lL) < L) ++lL;
        const int s1 = __builtin_ctz(h->nk[0]), s2 = __builtin_ctz(h->nk[1]), s3 = __builtin_ctz(h->nk[2]);
#define OCEAN_POW2_ARGS                                                                            \
    phi, W, ph, s1, s2, s3, h->nx[0], h->nx[1], h->nx[2], h->phase_off[0], h->phase_off[1],         \
        h->phase_off[2], (int)total, cols, lL, pad, phase
        if (nmax <= 2)
            fft_w_pow2_kernel<T, S, 2><<<nblk, 256, lds2, h->stream>>>(OCEAN_POW2_ARGS);
        else if (nmax <= 4)
            fft_w_pow2_kernel<T, S, 4><<<nblk, 256, lds2, h->stream>>>(OCEAN_POW2_ARGS);
        else if (nmax <= 8)
            fft_w_pow2_kernel<T, S, 8><<<nblk, 256, lds2, h->stream>>>(OCEAN_POW2_ARGS);
        else
            fft_w_pow2_kernel<T, S, 16><<<nblk, 256, lds2, h->stream>>>(OCEAN_POW2_ARGS);
#undef OCEAN_POW2_ARGS
        return hipGetLastError();
    }
#define OCEAN_FFT_ARGS                                                                          \
    phi, W, ph, tw, h->nk[0], h->nk[1], h->nk[2], h->nx[0], h->nx[1], h->nx[2], h->phase_off[0], \
        h->phase_off[1], h->phase_off[2], h->tw_off[0], h->tw_off[1], h->tw_off[2], h->Nx, cols, L, phase
    if (nmax <= 2)
        fft_w_kernel<T, S, 2><<<nblk, 256, lds, h->stream>>>(OCEAN_FFT_ARGS);
    else if (nmax <= 4)
        fft_w_kernel<T, S, 4><<<nblk, 256, lds, h->stream>>>(OCEAN_FFT_ARGS);
    else if (nmax <= 8)
        fft_w_kernel<T, S, 8><<<nblk, 256, lds, h->stream>>>(OCEAN_FFT_ARGS);
    else
        fft_w_kernel<T, S, 16><<<nblk, 256, lds, h->stream>>>(OCEAN_FFT_ARGS);
#undef OCEAN_FFT_ARGS
    return hipGetLastError();
}

}  // namespace

size_t fft_lds_bytes(const ocean_bse_s* h, int lines) {
    const size_t elem = h->precision == OCEAN_PREC_FP64 ? 16 : 8;
    if (cube_ok(h, lines)) {
        const int n = h->nk[0], M = 256 / (int)elem;
        const int pad = (M - ((n - 1) * lines) % M) % M;
        return elem * ((size_t)n * n * n * lines + (size_t)n * n * pad);
    }
    if (is_pow2_grid(h))
        return elem * ((size_t)h->Nk * lines + (size_t)(h->Nk / h->nk[2]) * pow2_pad((int)elem, h->nk[2], lines));
    return elem * (3 * kMaxDft + (size_t)h->Nk * lines);
}

hipError_t launch_fft_w(ocean_bse_s* h, int cols) {
    const int slot = prof_begin(h, "fft_w");
    hipError_t e;
    if (h->precision == OCEAN_PREC_FP64)
        e = fft_dispatch<double, double2>(h, cols, h->W64);
    else if (h->precision == OCEAN_PREC_BF16)
        e = fft_dispatch<float, bf16c>(h, cols, h->W32);
    else
        e = fft_dispatch<float, float2>(h, cols, h->W32);
    prof_end(h, slot);
    return e;
}

}  // namespace ocean
