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
// The pass is HBM-bound: phi is read once and written once.
#include "internal.h"

namespace ocean {
namespace {

template <typename T> struct C2T;
template <> struct C2T<double> { typedef double2 t; };
template <> struct C2T<float> { typedef float2 t; };

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
            v = phi[(size_t)kk * total + line];
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
            const T w = W[(size_t)x * Nk + r];
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
            phi[(size_t)kk * total + line] = cmul(buf[e], pc);
        }
    }
}

template <typename T>
hipError_t fft_dispatch(ocean_bse_s* h, int cols, const T* W) {
    typedef typename C2T<T>::t C2;
    const int L = h->fft_lines;
    const long long total = (long long)h->Nx * cols;
    const unsigned nblk = (unsigned)((total + L - 1) / L);
    const size_t lds = sizeof(C2) * (3 * kMaxDft + (size_t)h->Nk * L);
    const int nmax = std::max(h->nk[0], std::max(h->nk[1], h->nk[2]));
    C2* phi = static_cast<C2*>(h->ws.phi);
    const double2* ph = reinterpret_cast<const double2*>(h->phase);
    const double2* tw = reinterpret_cast<const double2*>(h->twiddle);
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
