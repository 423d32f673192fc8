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
// 8 contraction points, two per lane group, and each point feeds two MFMAs (re and im part);
// which two points a lane group holds is chosen per kernel so that its loads coalesce.
//
// On gfx950 an FP64 16x16x4 MFMA takes the issue slots of 16 wave-wide FP64 FMAs, so in FP64
// a pass whose columns leave at most 2 complex columns after whole 16-wide tiles contracts
// those with plain FMAs instead of a mostly empty tile.
#include <type_traits>

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

// f32 4x4x1 MFMA with 16 blocks: block b = lane / 4 computes D_b[r][j] += A_b[r] B_b[j] with A_b[r]
// the value of lane 4 b + r and B_b[j] that of lane 4 b + j; D_b[r][j] sits in lane 4 b + j,
// register r (measured on gfx950).  With the 16x16 operand layout (lane = i + 16 kq) a block is
// rows 4 (b % 4) .. +3 of lane group kq = b / 4, so one call contracts each lane group's own
// point for a 16-row by 4-column tile; the four lane groups are added at the end.  It runs at the
// matrix cores' full rate, so a 4-column remainder costs a quarter of a 16-column tile.
__device__ __forceinline__ v4f mfma_quad(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

template <typename T> struct Cplx;
template <> struct Cplx<double> { typedef double2 c2; typedef v4d acc; };
template <> struct Cplx<float> { typedef float2 c2; typedef v4f acc; };

// Row of the 16x16 result held in accumulator register r of a lane in group kq
// (column = lane % 16).  The f64 and f32 16x16x4 instructions differ here.
template <typename T> __device__ __forceinline__ int acc_row(int kq, int r);
template <> __device__ __forceinline__ int acc_row<double>(int kq, int r) { return 4 * r + kq; }
template <> __device__ __forceinline__ int acc_row<float>(int kq, int r) { return 4 * kq + r; }

// Forward projection: B operands are staged in LDS in MFMA order: value s (0..3) of lane l
// for sub-step ss and column tile t sits at ((ss * NT + t) * 64 + l) * 4 + s, so a wave reads
// its operands with one 4-wide LDS load per (ss, t).  Lane l = i + 16 kq of sub-step ss
// covers the bands fwd_band(kq, s / 2) of that 8-band step (parts s % 2) and real column
// 16 t + i.  FP64: the four lane groups take four consecutive bands (kq + 4 ns), so the 16-byte
// u loads of one row form one aligned 64-byte piece; FP32: a lane takes two consecutive bands
// (2 kq + ns) and loads both with one 16-byte load.
template <typename T> __device__ __forceinline__ int fwd_band(int kq, int ns) {
    return sizeof(T) == 8 ? kq + 4 * ns : 2 * kq + ns;
}

template <typename T> struct Vec4;
template <> struct Vec4<double> { typedef double4 t; };
template <> struct Vec4<float> { typedef float4 t; };

// Write the four B values [[re, im], [-im, re]] (rows p, columns q) of one complex psi value
// of band slot (kq, ns) of sub-step ss and local column cl into the MFMA-ordered buffer.
template <typename T, int NT>
__device__ __forceinline__ void stage_pair(T* buf, int ss, int kq, int ns, int cl, double re, double im) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int jr = 2 * cl + q;
        const int t = jr >> 4, i = jr & 15;
        if (t >= NT) continue;
        T* dst = buf + ((size_t)(ss * NT + t) * 64 + i + 16 * kq) * 4 + 2 * ns;
        dst[0] = (T)(q ? im : re);
        dst[1] = (T)(q ? re : -im);
    }
}

// ---------------------------------------------------------------------------------------------
// Forward projection.  Block = 4 waves and one k; wave w owns rows
// [xt*64*MS + w*16*MS, +16*MS) and every column tile.  The bands are walked in chunks of
// KC: the psi chunk (B operand, shared by all waves) is staged in LDS in MFMA order, double
// buffered, while each wave keeps the u values (A operand) of the next chunk in flight.  FP32
// runs a remainder of at most 4 real columns on the 4x4x1 MFMA (TQ = 1, as the resident form
// below does) instead of a mostly empty 16-column tile.
template <typename T, int MS, int NT, int TC, int TQ, int KC, int CP, bool PAIR>
__global__ __launch_bounds__(256) void proj_fwd_kernel(
    const typename Cplx<T>::c2* __restrict__ U, const double2* __restrict__ psi,
    typename Cplx<T>::c2* __restrict__ phi, int Nk, int Nx, int Nb, int Nc, int cols, int col0,
    int ncb, int x_tiles) {
    typedef typename Cplx<T>::c2 C2;
    typedef typename Cplx<T>::acc ACC;
    typedef typename Vec4<T>::t V4;
    constexpr int SS = KC / 8;                 // 8-band sub-steps per chunk
    constexpr int NS = NT + TQ;                // staged column tiles: the quad tail reads the last
    static_assert(TQ == 0 || sizeof(T) == 4, "quad tail: FP32");
    constexpr int BUF = SS * NS * 64 * 4;      // T values per staged chunk
    __shared__ __align__(16) T sB[2][BUF];
    __shared__ __align__(16) C2 sT[2][KC][TC > 0 ? TC : 1];   // FMA tail columns, (re, im)
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
    constexpr int PER = (KC * CP + 255) / 256;
    auto load_p = [&](int n0, double2 (&pv)[PER]) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = threadIdx.x + 256 * j;
            const int nl = e / CP, cl = e - nl * CP;
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
            const int nl = e / CP, cl = e - nl * CP;
            if (nl < KC && cl < ncb) {
                const int r8 = nl & 7;
                const int kq8 = sizeof(T) == 8 ? (r8 & 3) : (r8 >> 1), ns8 = sizeof(T) == 8 ? (r8 >> 2) : (r8 & 1);
                if (cl < 8 * NS) stage_pair<T, NS>(sB[buf], nl >> 3, kq8, ns8, cl, pv[j].x, pv[j].y);
                else if (TC > 0) sT[buf][nl][cl - 8 * NT] = C2{(T)pv[j].x, (T)pv[j].y};
            }
        }
    };
    auto load_a = [&](int n0, C2 (&aa)[MS][SS][2]) {
#pragma unroll
        for (int ss = 0; ss < SS; ++ss) {
            if constexpr (sizeof(T) == 8) {
#pragma unroll
                for (int ns = 0; ns < 2; ++ns) {
                    const int n = n0 + 8 * ss + fwd_band<T>(kq, ns);
                    const bool nok = n < Nb;
#pragma unroll
                    for (int ms = 0; ms < MS; ++ms)
                        aa[ms][ss][ns] = bload<C2>(ur, (nok && rval[ms]) ? urow[ms] + (unsigned)(n * sizeof(C2)) : kOob);
                }
            } else {
                // bands 2 kq and 2 kq + 1 in one 16-byte load (PAIR: Nb even; else two 8-byte
                // loads).  A compile-time choice: a branch here would merge two load counts and
                // make the compiler's waits for the ring's slots conservative.
                const int n = n0 + 8 * ss + 2 * kq;
#pragma unroll
                for (int ms = 0; ms < MS; ++ms) {
                    if constexpr (PAIR) {
                        const bool ok = n < Nb && rval[ms];
                        const float4 v = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(
                            ur, (int)(ok ? urow[ms] + (unsigned)(n * sizeof(C2)) : kOob), 0, 0));
                        aa[ms][ss][0] = C2{(T)v.x, (T)v.y};
                        aa[ms][ss][1] = C2{(T)v.z, (T)v.w};
                    } else {
#pragma unroll
                        for (int ns = 0; ns < 2; ++ns) {
                            const bool ok = n + ns < Nb && rval[ms];
                            aa[ms][ss][ns] = bload<C2>(ur, ok ? urow[ms] + (unsigned)((n + ns) * sizeof(C2)) : kOob);
                        }
                    }
                }
            }
        }
    };

    // padding columns stay zero in both buffers
    for (int e = threadIdx.x; e < 2 * BUF; e += 256) (&sB[0][0])[e] = (T)0;

    ACC acc[MS][NT];
#pragma unroll
    for (int ms = 0; ms < MS; ++ms)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[ms][t] = ACC{0, 0, 0, 0};
    // quad tail (FP32): the last <= 4 real columns on the 4x4x1 MFMA (the resident forward's
    // layout: lane l reads the B values lane (l % 4) + 16 kq holds for the staged tile NT)
    v4f accq[MS];
#pragma unroll
    for (int ms = 0; ms < MS; ++ms) accq[ms] = v4f{0.f, 0.f, 0.f, 0.f};
    const int qlane = (lane & 3) + (lane & 48);
    // FMA tail: lane (i, kq) sums its own bands for row i; the lane groups are added at the end
    T tre[MS][TC > 0 ? TC : 1], tim[MS][TC > 0 ? TC : 1];
#pragma unroll
    for (int ms = 0; ms < MS; ++ms)
#pragma unroll
        for (int c = 0; c < TC; ++c) tre[ms][c] = tim[ms][c] = (T)0;

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
                bv[t] = *reinterpret_cast<const V4*>(&sB[buf][((ss * NS + t) * 64 + lane) * 4]);
            V4 bq;
            if constexpr (TQ > 0) bq = *reinterpret_cast<const V4*>(&sB[buf][((ss * NS + NT) * 64 + qlane) * 4]);
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
                    if constexpr (TQ > 0) {
                        const T b = s == 0 ? bq.x : s == 1 ? bq.y : s == 2 ? bq.z : bq.w;
                        accq[ms] = mfma_quad((float)av, (float)b, accq[ms]);
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < TC; ++c)
#pragma unroll
                for (int ns = 0; ns < 2; ++ns) {
                    const C2 f = sT[buf][8 * ss + fwd_band<T>(kq, ns)][c];   // same address for the 16 lanes
#pragma unroll
                    for (int ms = 0; ms < MS; ++ms) {
                        const C2 v = a[ms][ss][ns];
                        tre[ms][c] = __builtin_fma(v.x, f.x, __builtin_fma(-v.y, f.y, tre[ms][c]));
                        tim[ms][c] = __builtin_fma(v.x, f.y, __builtin_fma(v.y, f.x, tim[ms][c]));
                    }
                }
        }
        // keep this chunk's tail sums here (sunk later they would pin the u registers)
#pragma unroll
        for (int ms = 0; ms < MS; ++ms)
#pragma unroll
            for (int c = 0; c < TC; ++c) asm volatile("" : "+v"(tre[ms][c]), "+v"(tim[ms][c]));
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
#pragma unroll
    for (int ms = 0; ms < MS; ++ms)
#pragma unroll
        for (int c = 0; c < TC; ++c) {
            T re = tre[ms][c], im = tim[ms][c];
            re += __shfl_xor(re, 16);
            im += __shfl_xor(im, 16);
            re += __shfl_xor(re, 32);
            im += __shfl_xor(im, 32);
            const int row = rowbase + 16 * ms + i;
            if (kq == 0 && row < Nx) {
                out[2 * phi_index_x(row, col0, k, Nk, cols) + 2 * (8 * NT + c)] = re;
                out[2 * phi_index_x(row, col0, k, Nk, cols) + 2 * (8 * NT + c) + 1] = im;
            }
        }
    if constexpr (TQ > 0) {
        // sum the lane groups; lane (i, kq) takes register r = kq: row 4 (i / 4) + kq, real
        // column 16 NT + i % 4; the even lane of each pair writes (re, im) of its complex column
#pragma unroll
        for (int ms = 0; ms < MS; ++ms) {
            v4f q4 = accq[ms];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                q4[r] += __shfl_xor(q4[r], 16);
                q4[r] += __shfl_xor(q4[r], 32);
            }
            const float q = kq == 0 ? q4[0] : kq == 1 ? q4[1] : kq == 2 ? q4[2] : q4[3];
            const float y = __shfl_xor(q, 1);
            const int c = 8 * NT + ((i & 3) >> 1);
            const int row = rowbase + 16 * ms + 4 * (i >> 2) + kq;
            if (!(lane & 1) && c < ncb && row < Nx) {
                out[2 * phi_index_x(row, col0 + c, k, Nk, cols)] = (T)q;
                out[2 * phi_index_x(row, col0 + c, k, Nk, cols) + 1] = (T)y;
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Forward projection with the B operand resident.  When every band of psi[k] fits in LDS (small
// band counts, such as 96 bands at the SrTiO3-shaped workload), a block stages psi[k] once, in
// the MFMA order above, and then streams u for `tiles` consecutive tiles of 16 * WAVES rows of
// that k.  Each wave owns 16 rows of every tile and walks its (tile, band chunk) items as one
// continuous pipeline: the u loads of the next RING - 1 items (the next chunks, running on into
// the next tile) are in flight while the current one is contracted.  After the staging there is
// no barrier, and a block starts once per `tiles` tiles instead of once per tile.
template <typename T, int NT, int TC, int TQ, int KC, int CP, int WAVES, int RING, bool PAIR>
__global__ __launch_bounds__(64 * WAVES) void proj_fwd_res_kernel(
    const typename Cplx<T>::c2* __restrict__ U, const double2* __restrict__ psi,
    typename Cplx<T>::c2* __restrict__ phi, int Nk, int Nx, int Nb, int Nc, int cols, int col0,
    int ncb, int groups, int tiles) {
    typedef typename Cplx<T>::c2 C2;
    typedef typename Cplx<T>::acc ACC;
    typedef typename Vec4<T>::t V4;
    constexpr int SS = KC / 8;
    constexpr int NTH = 64 * WAVES;
    constexpr int RPT = 16 * WAVES;            // rows per tile
    constexpr int NS = NT + TQ;                // staged column tiles: the quad tail reads the last
    static_assert(TQ == 0 || sizeof(T) == 4, "quad tail: FP32");
    static_assert(RING == 2 || RING == 3, "ring depth");
    extern __shared__ __align__(16) unsigned char smem[];
    const int nch = (Nb + KC - 1) / KC;
    T* sB = reinterpret_cast<T*>(smem);                                   // [nch SS][NS][64][4]
    C2* sT = reinterpret_cast<C2*>(sB + (size_t)nch * SS * NS * 256);     // [nch KC][TC]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const int k = blockIdx.x / groups;
    const int g = blockIdx.x - k * groups;
    const int x_tiles = (Nx + RPT - 1) / RPT;
    const int t0 = g * tiles, t1 = min(x_tiles, t0 + tiles);
    if (t0 >= t1) return;   // the whole block, before any barrier
    const C2* Uk = U + (size_t)k * Nx * Nb;
    const Rsrc ur = make_rsrc(Uk, (size_t)Nx * Nb * sizeof(C2));

    // psi[k], every band, in MFMA order; bands past Nb and padding columns stay zero
    const int nB = nch * SS * NS * 256;
    for (int e = threadIdx.x; e < nB; e += NTH) sB[e] = (T)0;
    if constexpr (TC > 0)
        for (int e = threadIdx.x; e < nch * KC * TC; e += NTH) sT[e] = C2{(T)0, (T)0};
    __syncthreads();
    for (int e = threadIdx.x; e < Nb * ncb; e += NTH) {
        const int n = e / ncb, cl = e - n * ncb;
        const int col = col0 + cl;
        const int vv = col / Nc, c = col - vv * Nc;
        const double2 pv = psi[(((size_t)vv * Nk + k) * Nb + n) * Nc + c];
        const int r8 = n & 7;
        const int kq8 = sizeof(T) == 8 ? (r8 & 3) : (r8 >> 1), ns8 = sizeof(T) == 8 ? (r8 >> 2) : (r8 & 1);
        if (cl < 8 * NS) stage_pair<T, NS>(sB, n >> 3, kq8, ns8, cl, pv.x, pv.y);
        else if constexpr (TC > 0) sT[n * TC + (cl - 8 * NT)] = C2{(T)pv.x, (T)pv.y};
    }
    __syncthreads();

    const int rowoff = wave * 16 + i;
    // quad tail: lane l takes real column 16 NT + l % 4 of its lane group, i.e. the B values
    // that lane (l % 4) + 16 kq holds for the staged tile NT
    const int qlane = (lane & 3) + (lane & 48);
    // u values of item (tile, chunk): lane (i, kq) holds row rowoff of the tile, the bands
    // fwd_band(kq, ns) of each 8-band sub-step; masked to zero past Nx, Nb or when !live
    auto load_a = [&](int tile, int ch, bool live, C2 (&aa)[SS][2]) {
        const int row = tile * RPT + rowoff;
        const bool rok = live && row < Nx;
        const unsigned rb = (unsigned)(row * Nb) * (unsigned)sizeof(C2);
        const int n0 = ch * KC;
#pragma unroll
        for (int ss = 0; ss < SS; ++ss) {
            if constexpr (sizeof(T) == 8) {
#pragma unroll
                for (int ns = 0; ns < 2; ++ns) {
                    const int n = n0 + 8 * ss + fwd_band<T>(kq, ns);
                    aa[ss][ns] = bload<C2>(ur, (rok && n < Nb) ? rb + (unsigned)(n * sizeof(C2)) : kOob);
                }
            } else {
                const int n = n0 + 8 * ss + 2 * kq;
                if constexpr (PAIR) {   // Nb even; see proj_fwd_kernel
                    const bool ok = rok && n < Nb;
                    const float4 v = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(
                        ur, (int)(ok ? rb + (unsigned)(n * sizeof(C2)) : kOob), 0, 0));
                    aa[ss][0] = C2{(T)v.x, (T)v.y};
                    aa[ss][1] = C2{(T)v.z, (T)v.w};
                } else {
#pragma unroll
                    for (int ns = 0; ns < 2; ++ns) {
                        const bool ok = rok && n + ns < Nb;
                        aa[ss][ns] = bload<C2>(ur, ok ? rb + (unsigned)((n + ns) * sizeof(C2)) : kOob);
                    }
                }
            }
        }
    };

    ACC acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = ACC{0, 0, 0, 0};
    v4f accq = {0.f, 0.f, 0.f, 0.f};
    T tre[TC > 0 ? TC : 1], tim[TC > 0 ? TC : 1];
#pragma unroll
    for (int c = 0; c < TC; ++c) tre[c] = tim[c] = (T)0;

    // the contraction of one item (the u values a of band chunk ch) against the resident psi[k]
    auto contract = [&](const C2 (&a)[SS][2], int ch) {
#pragma unroll
        for (int ss = 0; ss < SS; ++ss) {
            const int sg = ch * SS + ss;
            V4 bv[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) bv[t] = *reinterpret_cast<const V4*>(&sB[((sg * NS + t) * 64 + lane) * 4]);
            V4 bq;
            if constexpr (TQ > 0) bq = *reinterpret_cast<const V4*>(&sB[((sg * NS + NT) * 64 + qlane) * 4]);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const T av = (s & 1) ? a[ss][s >> 1].y : a[ss][s >> 1].x;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const T b = s == 0 ? bv[t].x : s == 1 ? bv[t].y : s == 2 ? bv[t].z : bv[t].w;
                    acc[t] = mfma16(av, b, acc[t]);
                }
                if constexpr (TQ > 0) {
                    const T b = s == 0 ? bq.x : s == 1 ? bq.y : s == 2 ? bq.z : bq.w;
                    accq = mfma_quad((float)av, (float)b, accq);
                }
            }
#pragma unroll
            for (int c = 0; c < TC; ++c)
#pragma unroll
                for (int ns = 0; ns < 2; ++ns) {
                    const C2 f = sT[(ch * KC + 8 * ss + fwd_band<T>(kq, ns)) * TC + c];   // same address for 16 lanes
                    const C2 v = a[ss][ns];
                    tre[c] = __builtin_fma(v.x, f.x, __builtin_fma(-v.y, f.y, tre[c]));
                    tim[c] = __builtin_fma(v.x, f.y, __builtin_fma(v.y, f.x, tim[c]));
                }
        }
#pragma unroll
        for (int c = 0; c < TC; ++c) asm volatile("" : "+v"(tre[c]), "+v"(tim[c]));
    };
    // tile done: write its 16 rows of phi and start the next one from zero.  FP64: each store
    // writes one complex value per lane: neighbouring lanes (real columns 2c and 2c + 1, the
    // re and im parts of complex column c) swap one of two accumulator rows, so that the even
    // lane holds column c of the first row and the odd lane column c of the second (half as
    // many store instructions as one real value per lane; the stores, not the bytes, cost).
    const Rsrc pw = make_rsrc(phi, phi_span_bytes(Nx, Nk, cols, (int)sizeof(C2)));
    const bool odd = lane & 1;
    auto finish_tile = [&](int tile) {
        const int rbase = tile * RPT + wave * 16;
        if constexpr (sizeof(T) == 4) {
            // FP32: two complex values per lane (shared with the bf16 forwards)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                store_fwd_tile<true>(acc[t], pw, 0, lane, rbase, 8 * t, Nx, ncb, col0, k, Nk, cols);
                acc[t] = ACC{0, 0, 0, 0};
            }
        } else {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = 8 * t + (i >> 1);   // this lane's complex column in the pass
#pragma unroll
            for (int rp = 0; rp < 2; ++rp) {
                const T a = acc[t][2 * rp], b = acc[t][2 * rp + 1];
                const T y = __shfl_xor(odd ? a : b, 1);
                const C2 v = odd ? C2{y, b} : C2{a, y};
                const int row = rbase + acc_row<T>(kq, 2 * rp + (odd ? 1 : 0));
                const bool ok = c < ncb && row < Nx;
                bstore<C2>(v, pw, ok ? (unsigned)(phi_index_x(row, col0 + c, k, Nk, cols) * sizeof(C2)) : kOob);
            }
            acc[t] = ACC{0, 0, 0, 0};
        }
        }
        if constexpr (TQ > 0) {
            // sum the lane groups (every group then holds the sums); lane (i, kq) takes
            // register r = kq: rows 4 (i / 4) + kq, real column 16 NT + i % 4
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                accq[r] += __shfl_xor(accq[r], 16);
                accq[r] += __shfl_xor(accq[r], 32);
            }
            const float q = kq == 0 ? accq[0] : kq == 1 ? accq[1] : kq == 2 ? accq[2] : accq[3];
            const float y = __shfl_xor(q, 1);
            const int c = 8 * NT + ((i & 3) >> 1);
            const int row = rbase + 4 * (i >> 2) + kq;
            const bool ok = !odd && c < ncb && row < Nx;
            bstore<C2>(C2{(T)q, (T)y}, pw, ok ? (unsigned)(phi_index_x(row, col0 + c, k, Nk, cols) * sizeof(C2)) : kOob);
            accq = v4f{0.f, 0.f, 0.f, 0.f};
        }
        if constexpr (TC > 0) {
            // every lane holds the sums after the butterfly; lane group kq writes tail column kq
            T re[TC], im[TC];
#pragma unroll
            for (int c = 0; c < TC; ++c) {
                re[c] = tre[c];
                im[c] = tim[c];
                re[c] += __shfl_xor(re[c], 16);
                im[c] += __shfl_xor(im[c], 16);
                re[c] += __shfl_xor(re[c], 32);
                im[c] += __shfl_xor(im[c], 32);
                tre[c] = tim[c] = (T)0;
            }
            C2 v = C2{re[0], im[0]};
#pragma unroll
            for (int c = 1; c < TC; ++c)
                if (kq == c) v = C2{re[c], im[c]};
            const int row = rbase + i;
            const bool ok = kq < TC && row < Nx;
            bstore<C2>(v, pw, ok ? (unsigned)(phi_index_x(row, col0 + 8 * NT + kq, k, Nk, cols) * sizeof(C2)) : kOob);
        }
    };

    // Items are (tile, chunk) pairs in order: (t0, 0), (t0, 1), .., (t1 - 1, nch - 1).  A ring
    // of RING register slots: while one item is contracted, the loads of the next RING - 1 are
    // in flight.  The ring is unrolled by its length so every slot is a static register set;
    // loads past the last item are masked (no memory access) and a turn has no exit between
    // its steps.
    int ct = t0, cc = 0;          // the item contracted next
    int lt = t0, lc = 0;          // the item loaded next
    auto advance = [&](int& t, int& c) {
        if (++c == nch) {
            c = 0;
            ++t;
        }
    };
    auto step = [&](const C2 (&cur)[SS][2], C2 (&nxt)[SS][2]) {
        load_a(lt, lc, lt < t1, nxt);
        advance(lt, lc);
        __builtin_amdgcn_sched_barrier(0);
        if (ct < t1) {
            contract(cur, cc);
            if (cc == nch - 1) finish_tile(ct);
            advance(ct, cc);
        }
    };
    const int n_items = (t1 - t0) * nch;
    C2 s0[SS][2], s1[SS][2];
    load_a(lt, lc, true, s0);
    advance(lt, lc);
    if constexpr (RING == 2) {
        for (int j = 0; j < n_items; j += 2) {
            step(s0, s1);
            step(s1, s0);
        }
    } else {
        C2 s2[SS][2];
        // FP32: keep the first two items' loads in item order, so that the compiler's waits at
        // the loop head count the second item's loads as still in flight (measured: FP32
        // faster, FP64 0.4% slower with the same ordering)
        if constexpr (sizeof(T) == 4) __builtin_amdgcn_sched_barrier(0);
        load_a(lt, lc, lt < t1, s1);
        advance(lt, lc);
        for (int j = 0; j < n_items; j += 3) {
            step(s0, s2);
            step(s1, s0);
            step(s2, s1);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);   // retire the masked loads past the last item before the exit
}

// ---------------------------------------------------------------------------------------------
// Backward projection with split-K over x.  Block = (k, band block of W x 16 bands,
// x chunk); wave w owns the 16 bands [band block * 16 W + 16 w, +16).  The chunk is walked
// in tiles of XT points through a ring of R slots: while tile t is contracted, the u values
// and the phi' values of tiles up to t + R - 1 are in flight (R = 3: 16-point tiles in FP64,
// 32-point tiles in FP32).  phi' tiles (shared by all waves) sit in
// LDS as [sub-step][lane group kq][column][q][point pair] complex pairs, q = 0 holding
// (re, im) and q = 1 holding (im, -re): the B operands of real column (column, q) are then
// the two halves of one pair, and a lane picks its orientation by address, with no per-lane
// select.
//
// Columns [0, 8 NT) go through NT MFMA column tiles.  The last TC (0..2; up to 4 in a wide
// pass) columns, which would fill at most a quarter (half) of one more tile, are contracted
// with plain FMAs instead: a 16x16x4 FP64 MFMA costs the issue slots of 16 wave-wide FMAs,
// so a tile holding 4 real columns of 16 wastes three quarters of them.  Lane (i, kq) sums
// its own points for band i, and the four lane groups are added at the end.
template <typename T, int NT, int TC, int TQ, int XT, int R, int W, int CP>
__global__ __launch_bounds__(64 * W) void proj_bwd_kernel(
    const typename Cplx<T>::c2* __restrict__ U, const typename Cplx<T>::c2* __restrict__ phi,
    double* __restrict__ part, int Nk, int Nx, int Nb, int cols, int col0, int ncb,
    int band_blocks, int S, int chunk) {
    typedef typename Cplx<T>::c2 C2;
    typedef typename Cplx<T>::acc ACC;
    constexpr int SS = XT / 8;
    constexpr int TILE = 2 * XT * CP;          // complex pairs of one phi' tile
    // phi' registers: FP64 one complex value per load; FP32 two adjacent columns per 16-byte
    // load (half the load instructions for the same bytes)
    constexpr int VC = sizeof(T) == 4 ? 2 : 1;
    typedef typename std::conditional<sizeof(T) == 4, float4, C2>::type PV;
    constexpr int CPV = CP / VC;               // loads per point
    static_assert(CP % VC == 0, "column pairs");
    constexpr int PER = (XT * CPV + 64 * W - 1) / (64 * W);
    static_assert(8 * NT + TC + 2 * TQ <= CP, "columns per pass");
    static_assert(R == 2 || R == 3, "ring depth");
    static_assert(TQ == 0 || sizeof(T) == 4, "quad tail: FP32");
    __shared__ __align__(16) C2 sP[R][TILE];
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
    const C2* Uk = U + (size_t)k * Nx * Nb;

    const int n = nbase + i;
    const bool nval = n < Nb;
    // u rows [x_begin, x_end) of this k, all bands; phi' x-blocks covering the chunk
    const Rsrc ur = make_rsrc(Uk + (size_t)x_begin * Nb, (size_t)(x_end - x_begin) * Nb * sizeof(C2));
    const int xb0 = x_begin / kXB;
    const C2* pbase = phi + (size_t)xb0 * Nk * kXB * cols;
    const Rsrc prs = make_rsrc(pbase, (size_t)((x_end - 1) / kXB - xb0 + 1) * Nk * kXB * cols * sizeof(C2));

    // tile loads (masked to zero past the chunk end)
    auto issue = [&](int x0, PV (&pp)[PER], C2 (&uu)[SS][2]) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = threadIdx.x + 64 * W * j;
            const int xl = e / CPV, cl = VC * (e - xl * CPV);
            const int x = x0 + xl;
            const bool ok = xl < XT && cl < ncb && x < x_end;
            const unsigned off = (unsigned)((phi_index_x(x, col0 + cl, k, Nk, cols) - (size_t)xb0 * Nk * kXB * cols) * sizeof(C2));
            if constexpr (VC == 2) {
                float4 v = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(prs, (int)(ok ? off : kOob), 0, 0));
                if (cl + 1 >= ncb) v.z = v.w = 0.f;   // past the pass: the next point's column, or nothing
                pp[j] = v;
            } else {
                pp[j] = bload<C2>(prs, ok ? off : kOob);
            }
        }
#pragma unroll
        for (int ss = 0; ss < SS; ++ss)
#pragma unroll
            for (int xs = 0; xs < 2; ++xs) {
                const int x = x0 + 8 * ss + 2 * kq + xs;
                const bool ok = nval && x < x_end;
                uu[ss][xs] = bload_stream<C2>(ur, ok ? (unsigned)(((x - x_begin) * Nb + n) * sizeof(C2)) : kOob);
            }
    };
    // point xl of the tile = (sub-step xl / 8, lane group (xl % 8) / 2, pair slot xl % 2)
    auto stage = [&](C2* dst, const PV (&pp)[PER]) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = threadIdx.x + 64 * W * j;
            const int xl = e / CPV, cl0 = VC * (e - xl * CPV);
#pragma unroll
            for (int q = 0; q < VC; ++q) {
                const int cl = cl0 + q;
                if (xl < XT && cl < ncb) {
                    C2 v;
                    if constexpr (VC == 2) v = q ? C2{pp[j].z, pp[j].w} : C2{pp[j].x, pp[j].y};
                    else v = pp[j];
                    C2* d = dst + ((((xl >> 3) * 4 + ((xl & 7) >> 1)) * CP + cl) * 2) * 2 + (xl & 1);
                    d[0] = v;
                    d[2] = C2{v.y, -v.x};
                }
            }
        }
    };
    ACC acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = ACC{0, 0, 0, 0};
    T tre[TC > 0 ? TC : 1], tim[TC > 0 ? TC : 1];
#pragma unroll
    for (int c = 0; c < TC; ++c) tre[c] = tim[c] = (T)0;
    v4f accq = {0.f, 0.f, 0.f, 0.f};
    // quad tail: lane l takes real column 16 NT + l % 4, i.e. (column 8 NT + (l % 4) / 2, q = l % 2)
    const int qoff = (8 * NT + ((lane & 3) >> 1)) * 4 + (lane & 1) * 2;
    auto contract = [&](const C2* src, const C2 (&uu)[SS][2]) {
#pragma unroll
        for (int ss = 0; ss < SS; ++ss) {
            const C2* row = src + (ss * 4 + kq) * CP * 4;
            // lane (i, kq): real column (8 t + i / 2, q = i % 2) -> pair (column, q)
            const C2* mine = row + (i >> 1) * 4 + (i & 1) * 2;
            C2 b[NT][2];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                b[t][0] = mine[32 * t];
                b[t][1] = mine[32 * t + 1];
            }
            C2 bq[2];
            if constexpr (TQ > 0) {
                bq[0] = row[qoff];
                bq[1] = row[qoff + 1];
            }
#pragma unroll
            for (int xs = 0; xs < 2; ++xs) {
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = mfma16(uu[ss][xs].x, b[t][xs].x, acc[t]);
                if constexpr (TQ > 0) accq = mfma_quad((float)uu[ss][xs].x, (float)bq[xs].x, accq);
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = mfma16(uu[ss][xs].y, b[t][xs].y, acc[t]);
                if constexpr (TQ > 0) accq = mfma_quad((float)uu[ss][xs].y, (float)bq[xs].y, accq);
            }
#pragma unroll
            for (int c = 0; c < TC; ++c)
#pragma unroll
                for (int xs = 0; xs < 2; ++xs) {
                    const C2 f = row[(8 * NT + c) * 4 + xs];   // (re, im); same address for the 16 lanes
                    const C2 v = uu[ss][xs];
                    tre[c] = __builtin_fma(v.x, f.x, __builtin_fma(v.y, f.y, tre[c]));
                    tim[c] = __builtin_fma(v.x, f.y, __builtin_fma(-v.y, f.x, tim[c]));
                }
        }
        // keep the tail sums of this tile here: sunk into a later step they would hold this
        // tile's u registers past the loads that reuse them
#pragma unroll
        for (int c = 0; c < TC; ++c) asm volatile("" : "+v"(tre[c]), "+v"(tim[c]));
    };

    // padding columns stay zero in every buffer
    for (int e = threadIdx.x; e < R * TILE; e += 64 * W) (&sP[0][0])[e] = C2{0, 0};

    C2 ua[R][SS][2];
    PV pr[R][PER];
#pragma unroll
    for (int r = 0; r + 1 < R; ++r) issue(x_begin + r * XT, pr[r], ua[r]);
    __syncthreads();
    stage(sP[0], pr[0]);
    // step on tile x0 held in ring slot c: request tile x0 + (R - 1) XT into slot c + R - 1,
    // contract slot c, stage tile x0 + XT (slot c + 1) into its LDS buffer.  The barrier at
    // the top publishes the previous step's staging and retires every read of the buffer
    // staged now.
    auto step = [&](int x0, PV (&pn)[PER], C2 (&un)[SS][2], const C2* cur, const C2 (&uc)[SS][2],
                    C2* nxt, const PV (&p1)[PER]) {
        __syncthreads();
        issue(x0 + (R - 1) * XT, pn, un);
        __builtin_amdgcn_sched_barrier(0);
        contract(cur, uc);
        stage(nxt, p1);
    };
    // whole turns of the ring (tiles past the chunk end are zero): no exit between steps, so
    // every step sees the same loads outstanding
    if constexpr (R == 3) {
        for (int x0 = x_begin; x0 < x_end; x0 += 3 * XT) {
            step(x0, pr[2], ua[2], sP[0], ua[0], sP[1], pr[1]);
            step(x0 + XT, pr[0], ua[0], sP[1], ua[1], sP[2], pr[2]);
            step(x0 + 2 * XT, pr[1], ua[1], sP[2], ua[2], sP[0], pr[0]);
        }
    } else {
        for (int x0 = x_begin; x0 < x_end; x0 += 2 * XT) {
            step(x0, pr[1], ua[1], sP[0], ua[0], sP[1], pr[1]);
            step(x0 + XT, pr[0], ua[0], sP[1], ua[1], sP[0], pr[0]);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);   // retire the loads past the chunk end before the exit

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
#pragma unroll
    for (int c = 0; c < TC; ++c) {
        T re = tre[c], im = tim[c];
        re += __shfl_xor(re, 16);
        im += __shfl_xor(im, 16);
        re += __shfl_xor(re, 32);
        im += __shfl_xor(im, 32);
        if (kq == 0 && nval) {
            out[(size_t)n * 2 * cols + 2 * (8 * NT + c)] = (double)re;
            out[(size_t)n * 2 * cols + 2 * (8 * NT + c) + 1] = (double)im;
        }
    }
    if constexpr (TQ > 0) {
        // sum the lane groups; lane l < 16 then holds bands 4 (l / 4) + r, real column 16 NT + l % 4
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            accq[r] += __shfl_xor(accq[r], 16);
            accq[r] += __shfl_xor(accq[r], 32);
        }
        const int jr = 16 * NT + (lane & 3);
        if (kq == 0 && (jr >> 1) < ncb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int nn = nbase + 4 * (lane >> 2) + r;
                if (nn < Nb) out[(size_t)nn * 2 * cols + jr] = (double)accq[r];
            }
        }
    }
}

// KC: bands per forward chunk; XT, R: back-projection x tile and ring depth; RR: ring depth of
// the resident forward (two items in flight while one is contracted)
template <typename T> struct Tiles;
template <> struct Tiles<double> { static constexpr int KC = 16, XT = 16, R = 3, RR = 3; };
template <> struct Tiles<float> { static constexpr int KC = 32, XT = 32, R = 3, RR = 3; };

template <typename T, int MS>
hipError_t fwd_dispatch_nt(int NT, int TC, int TQ, dim3 grid, hipStream_t st, const void* U, const double* x,
                           void* phi, int Nk, int Nx, int Nb, int Nc, int cols, int col0, int ncb,
                           int x_tiles) {
    typedef typename Cplx<T>::c2 C2;
    const C2* u = static_cast<const C2*>(U);
    C2* p = static_cast<C2*>(phi);
    const double2* ps = reinterpret_cast<const double2*>(x);
    // FP32 with an even band count loads two bands per 16-byte load (PAIR)
    const bool pair = sizeof(T) == 4 && (Nb & 1) == 0;
#define OCEAN_FWD(nt, tc, tq, cp) \
    if (NT == nt && TC == tc && TQ == tq) { \
        if (pair) \
            proj_fwd_kernel<T, MS, nt, tc, tq, Tiles<T>::KC, cp, sizeof(T) == 4><<<grid, 256, 0, st>>>(u, ps, p, Nk, Nx, Nb, Nc, cols, col0, ncb, x_tiles); \
        else \
            proj_fwd_kernel<T, MS, nt, tc, tq, Tiles<T>::KC, cp, false><<<grid, 256, 0, st>>>(u, ps, p, Nk, Nx, Nb, Nc, cols, col0, ncb, x_tiles); \
        return hipGetLastError(); \
    }
    if (ncb <= kColsPerPass) {
        OCEAN_FWD(1, 0, 0, kColsPerPass) OCEAN_FWD(2, 0, 0, kColsPerPass) OCEAN_FWD(3, 0, 0, kColsPerPass)
        if constexpr (sizeof(T) == 8) {
            OCEAN_FWD(1, 1, 0, kColsPerPass) OCEAN_FWD(1, 2, 0, kColsPerPass)
            OCEAN_FWD(2, 1, 0, kColsPerPass) OCEAN_FWD(2, 2, 0, kColsPerPass)
        } else {
            OCEAN_FWD(1, 0, 1, kColsPerPass) OCEAN_FWD(2, 0, 1, kColsPerPass)
        }
    } else if constexpr (sizeof(T) == 8 && MS == 1) {
        OCEAN_FWD(3, 1, 0, kColsPerWidePass) OCEAN_FWD(3, 2, 0, kColsPerWidePass) OCEAN_FWD(4, 0, 0, kColsPerWidePass)
        OCEAN_FWD(4, 1, 0, kColsPerWidePass) OCEAN_FWD(4, 2, 0, kColsPerWidePass) OCEAN_FWD(5, 0, 0, kColsPerWidePass)
    }
#undef OCEAN_FWD
    return hipErrorInvalidValue;
}

constexpr int kResWaves = 8;

template <typename T>
hipError_t fwd_res_dispatch(int NT, int TC, int TQ, dim3 grid, size_t lds, hipStream_t st, const void* U,
                            const double* x, void* phi, int Nk, int Nx, int Nb, int Nc, int cols, int col0,
                            int ncb, int groups, int tiles) {
    constexpr int KC = Tiles<T>::KC;
    typedef typename Cplx<T>::c2 C2;
    const C2* u = static_cast<const C2*>(U);
    C2* p = static_cast<C2*>(phi);
    const double2* ps = reinterpret_cast<const double2*>(x);
    const bool pair = sizeof(T) == 4 && (Nb & 1) == 0;
#define OCEAN_FWDR(nt, tc, tq) \
    if (NT == nt && TC == tc && TQ == tq) { \
        if (pair) \
            proj_fwd_res_kernel<T, nt, tc, tq, KC, kColsPerPass, kResWaves, Tiles<T>::RR, sizeof(T) == 4> \
                <<<grid, 64 * kResWaves, lds, st>>>(u, ps, p, Nk, Nx, Nb, Nc, cols, col0, ncb, groups, tiles); \
        else \
            proj_fwd_res_kernel<T, nt, tc, tq, KC, kColsPerPass, kResWaves, Tiles<T>::RR, false> \
                <<<grid, 64 * kResWaves, lds, st>>>(u, ps, p, Nk, Nx, Nb, Nc, cols, col0, ncb, groups, tiles); \
        return hipGetLastError(); \
    }
    OCEAN_FWDR(1, 0, 0) OCEAN_FWDR(2, 0, 0) OCEAN_FWDR(3, 0, 0)
    if constexpr (sizeof(T) == 8) {
        OCEAN_FWDR(1, 1, 0) OCEAN_FWDR(1, 2, 0) OCEAN_FWDR(2, 1, 0) OCEAN_FWDR(2, 2, 0)
    } else {
        OCEAN_FWDR(1, 0, 1) OCEAN_FWDR(2, 0, 1)
    }
#undef OCEAN_FWDR
    return hipErrorInvalidValue;
}


template <typename T, int W>
hipError_t bwd_dispatch_w(int NT, int TC, int TQ, dim3 grid, hipStream_t st, const void* U, const void* phi,
                          double* part, int Nk, int Nx, int Nb, int cols, int col0, int ncb, int bb,
                          int S, int chunk) {
    typedef typename Cplx<T>::c2 C2;
    constexpr int XT = Tiles<T>::XT;
    const C2* u = static_cast<const C2*>(U);
    const C2* p = static_cast<const C2*>(phi);
#define OCEAN_BWDQ(nt, tc, tq, cp) \
    if (NT == nt && TC == tc && TQ == tq) { \
        proj_bwd_kernel<T, nt, tc, tq, XT, Tiles<T>::R, W, cp><<<grid, 64 * W, 0, st>>>(u, p, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk); \
        return hipGetLastError(); \
    }
#define OCEAN_BWD(nt, tc, cp) OCEAN_BWDQ(nt, tc, 0, cp)
    if (ncb <= kColsPerPass) {
        OCEAN_BWD(1, 0, kColsPerPass) OCEAN_BWD(2, 0, kColsPerPass) OCEAN_BWD(3, 0, kColsPerPass)
        if constexpr (sizeof(T) == 8) {
            OCEAN_BWD(1, 1, kColsPerPass) OCEAN_BWD(1, 2, kColsPerPass)
            OCEAN_BWD(2, 1, kColsPerPass) OCEAN_BWD(2, 2, kColsPerPass)
        } else {
            OCEAN_BWDQ(1, 0, 1, kColsPerPass) OCEAN_BWDQ(2, 0, 1, kColsPerPass)
        }
    } else if constexpr (sizeof(T) == 8) {
        OCEAN_BWD(3, 1, kColsPerWidePass) OCEAN_BWD(3, 2, kColsPerWidePass) OCEAN_BWD(3, 3, kColsPerWidePass)
        OCEAN_BWD(3, 4, kColsPerWidePass) OCEAN_BWD(4, 0, kColsPerWidePass) OCEAN_BWD(4, 1, kColsPerWidePass)
        OCEAN_BWD(4, 2, kColsPerWidePass) OCEAN_BWD(4, 3, kColsPerWidePass) OCEAN_BWD(4, 4, kColsPerWidePass)
        OCEAN_BWD(5, 0, kColsPerWidePass)
    }
#undef OCEAN_BWD
#undef OCEAN_BWDQ
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t bwd_dispatch(int W, int NT, int TC, int TQ, dim3 grid, hipStream_t st, const void* U, const void* phi,
                        double* part, int Nk, int Nx, int Nb, int cols, int col0, int ncb, int bb,
                        int S, int chunk) {
    switch (W) {
#define OCEAN_BWD_W(w) \
        case w: return bwd_dispatch_w<T, w>(NT, TC, TQ, grid, st, U, phi, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk);
        OCEAN_BWD_W(1) OCEAN_BWD_W(2) OCEAN_BWD_W(3) OCEAN_BWD_W(4) OCEAN_BWD_W(5) OCEAN_BWD_W(6)
        OCEAN_BWD_W(7)
#undef OCEAN_BWD_W
        default: return bwd_dispatch_w<T, 8>(NT, TC, TQ, grid, st, U, phi, part, Nk, Nx, Nb, cols, col0, ncb, bb, S, chunk);
    }
}

}  // namespace


// Backward-projection geometry: band blocks of at most `cap` waves x 16 bands, the 16-band
// groups dealt evenly over the fewest blocks (96 bands at cap 4: two blocks of 3 waves), and x
// chunks (multiples of the 16-point phi x-block) so that the grid holds about
// bwd_target_blocks blocks.
int bwd_waves_for(int Nb, int cap) {
    const int nb16 = (Nb + 15) / 16;
    const int blocks = (nb16 + cap - 1) / cap;
    return (nb16 + blocks - 1) / blocks;
}

int bwd_waves(const ocean_bse_s* h) { return bwd_waves_for(h->Nb, h->bwd_waves); }

void bwd_geometry_for(const ocean_bse_s* h, int target_blocks, int W, int* band_blocks, int* S, int* chunk) {
    const int bb = (h->Nb + 16 * W - 1) / (16 * W);
    const long long per_chunk = (long long)h->Nk * bb;
    long long s = (target_blocks + per_chunk - 1) / per_chunk;
    const long long smax = std::max(1, (h->Nx + 511) / 512);  // >= 512 points per chunk
    // The partials of one chunk (kColsPerPass complex FP64 columns per band; a wide FP64 pass
    // writes 5/3 of that) written and read back stay within 5% of the u bytes the chunk streams.  This binds for
    // Gamma-only systems with many x points, whose grid otherwise comes from x chunks alone.
    const int ue = h->precision == OCEAN_PREC_FP64 ? 16 : h->precision == OCEAN_PREC_BF16 ? 4 : 8;
    const long long scap = std::max(1LL, (long long)h->Nx * ue / (20LL * 16 * kColsPerPass));
    if (s < 1) s = 1;
    if (s > smax) s = smax;
    if (s > scap) s = scap;
    int c = (int)((h->Nx + s - 1) / s);
    c = (c + kXB - 1) / kXB * kXB;
    *chunk = c;
    *S = (h->Nx + c - 1) / c;
    *band_blocks = bb;
}

void bwd_geometry(const ocean_bse_s* h, int* band_blocks, int* S, int* chunk) {
    bwd_geometry_for(h, h->bwd_target_blocks, bwd_waves(h), band_blocks, S, chunk);
}

bool is_bf16_mode(int precision) {
    return precision == OCEAN_PREC_SPLIT_BF16 || precision == OCEAN_PREC_BF16;
}

int fwd_band_chunk(const ocean_bse_s* h) { return is_bf16_mode(h->precision) ? 32 : 0; }

// Columns per projection launch: every pass streams all of u once, so FP64 runs up to
// kColsPerWidePass columns (five MFMA column tiles, or four and the FMA tail) in one pass,
// e.g. the 36 columns of three polarisations with the electron and hole spins separate.
// The other precisions keep kColsPerPass.
int cols_per_pass(const ocean_bse_s* h, int cols) {
    return h->precision == OCEAN_PREC_FP64 && cols > kColsPerPass && cols <= kColsPerWidePass ? kColsPerWidePass
                                                                                            : kColsPerPass;
}

// MFMA column tiles and FMA tail columns for ncb complex columns.  In FP64 a remainder of at
// most 4 real columns (2 complex) after whole 16-wide tiles goes to the FMA tail; FP32 MFMAs
// are cheap next to FP32 FMAs, so FP32 always rounds up to whole tiles.
// A wide FP64 back-projection (more than kColsPerPass columns) is bound by the matrix cores
// rather than by HBM; there the tail takes up to 4 columns, so the 36 columns of the full
// spin space use four tiles and a 4-column tail rather than five tiles (measured: 2.56
// against 2.71 ms at 36 columns).  The wide forward keeps the 2-column limit: with a
// 4-column tail it needs 182 VGPRs, one wave per SIMD fewer, and was slower (2.66 against
// 2.50 ms).
// With quad (FP32 kernels that have it), a remainder of at most 4 real columns after whole
// tiles goes to the 4x4x1 quad tail instead (TQ = 1), at the matrix cores' full rate.
void column_split(int ncb, bool fp64, bool wide_tail, bool quad, int* NT, int* TC, int* TQ) {
    const int full = 2 * ncb / 16, rem = 2 * ncb - 16 * full;
    const int max_tail = wide_tail && ncb > kColsPerPass ? 8 : 4;   // real columns
    *TQ = 0;
    if (rem == 0) { *NT = full; *TC = 0; }
    else if (fp64 && rem <= max_tail && full >= 1) { *NT = full; *TC = rem / 2; }
    else if (!fp64 && quad && rem <= 4 && full >= 1) { *NT = full; *TC = 0; *TQ = 1; }
    else { *NT = full + 1; *TC = 0; }
}

// LDS bytes of the resident-operand forward for a pass of ncb columns, or 0 if psi[k] of every
// band does not fit in 64 KiB (or the pass is wide, or one k of u spans more than 2 GiB, or in
// FP64/FP32 phi spans 4 GiB or more).
size_t fwd_res_lds_bytes(const ocean_bse_s* h, int ncb) {
    if (ncb > kColsPerPass) return 0;
    if (is_bf16_mode(h->precision)) {
        // the staged B chunks of every band (both planes), 4 KiB per chunk and column tile
        const size_t NT = (2 * ncb + 15) / 16;
        const int KC = fwd_band_chunk(h);
        const size_t b = (size_t)((h->Nb + KC - 1) / KC) * NT * kStageTile;
        if ((size_t)h->Nx * h->Nb * 4 >= (1ull << 31)) return 0;
        return b <= 64 * 1024 ? b : 0;
    }
    const bool fp64 = h->precision == OCEAN_PREC_FP64;
    int NT, TC, TQ;
    column_split(ncb, fp64, false, true, &NT, &TC, &TQ);
    const size_t elem = fp64 ? 8 : 4;
    const int KC = fp64 ? Tiles<double>::KC : Tiles<float>::KC;
    const size_t nch = (h->Nb + KC - 1) / KC;
    if ((size_t)h->Nx * h->Nb * 2 * elem >= (1ull << 31)) return 0;
    // phi is written through a buffer descriptor with 32-bit byte offsets
    const size_t nx_pad = ((size_t)h->Nx + kXB - 1) / kXB * kXB;
    if ((size_t)h->Nk * nx_pad * std::max(h->ws.cols, ncb) * 2 * elem >= kOob) return 0;
    const size_t b = nch * (KC / 8) * (NT + TQ) * 256 * elem + nch * KC * TC * 2 * elem;
    return b <= 64 * 1024 ? b : 0;
}

hipError_t launch_proj_fwd(ocean_bse_s* h, const double* x, int nv, int col0, int ncb) {
    if (is_bf16_mode(h->precision)) return launch_proj_fwd_bf16(h, x, nv, col0, ncb);
    if (h->fwd_tiles > 0) {
        const size_t lds = fwd_res_lds_bytes(h, ncb);
        if (lds > 0) {
            int NT, TC, TQ;
            column_split(ncb, h->precision == OCEAN_PREC_FP64, false, h->quad_tail != 0, &NT, &TC, &TQ);
            const int rpt = 16 * kResWaves;
            const int x_tiles = (h->Nx + rpt - 1) / rpt;
            const int tiles = std::min(h->fwd_tiles, x_tiles);
            const int groups = (x_tiles + tiles - 1) / tiles;
            dim3 grid((unsigned)((long long)h->Nk * groups));
            const int slot = prof_begin(h, "proj_fwd");
            hipError_t e;
            if (h->precision == OCEAN_PREC_FP64)
                e = fwd_res_dispatch<double>(NT, TC, TQ, grid, lds, h->stream, h->U64, x, h->ws.phi, h->Nk, h->Nx,
                                             h->Nb, h->Nc, nv * h->Nc, col0, ncb, groups, tiles);
            else
                e = fwd_res_dispatch<float>(NT, TC, TQ, grid, lds, h->stream, h->U32, x, h->ws.phi, h->Nk, h->Nx,
                                            h->Nb, h->Nc, nv * h->Nc, col0, ncb, groups, tiles);
            prof_end(h, slot);
            return e;
        }
    }
    // 16 * MS rows per wave, 64 * MS per block; a wide pass (more than kColsPerPass columns)
    // holds more accumulators per wave and runs with MS = 1
    const int MS = (h->fwd_ms == 1 || ncb > kColsPerPass) ? 1 : 2;
    const int cols = nv * h->Nc;
    int NT, TC, TQ;
    column_split(ncb, h->precision == OCEAN_PREC_FP64, false, h->quad_tail != 0, &NT, &TC, &TQ);
    const int x_tiles = (h->Nx + 64 * MS - 1) / (64 * MS);
    dim3 grid((unsigned)(h->Nk * x_tiles));
    hipError_t e;
    const int slot = prof_begin(h, "proj_fwd");
    if (h->precision == OCEAN_PREC_FP64)
        e = MS == 1 ? fwd_dispatch_nt<double, 1>(NT, TC, TQ, grid, h->stream, h->U64, x, h->ws.phi, h->Nk, h->Nx,
                                                 h->Nb, h->Nc, cols, col0, ncb, x_tiles)
                    : fwd_dispatch_nt<double, 2>(NT, TC, TQ, grid, h->stream, h->U64, x, h->ws.phi, h->Nk, h->Nx,
                                                 h->Nb, h->Nc, cols, col0, ncb, x_tiles);
    else
        e = MS == 1 ? fwd_dispatch_nt<float, 1>(NT, TC, TQ, grid, h->stream, h->U32, x, h->ws.phi, h->Nk, h->Nx,
                                                h->Nb, h->Nc, cols, col0, ncb, x_tiles)
                    : fwd_dispatch_nt<float, 2>(NT, TC, TQ, grid, h->stream, h->U32, x, h->ws.phi, h->Nk, h->Nx,
                                                h->Nb, h->Nc, cols, col0, ncb, x_tiles);
    prof_end(h, slot);
    return e;
}

hipError_t launch_proj_bwd(ocean_bse_s* h, int nv, int col0, int ncb) {
    if (is_bf16_mode(h->precision)) return launch_proj_bwd_bf16(h, nv, col0, ncb);
    const int cols = nv * h->Nc;
    int NT, TC, TQ;
    column_split(ncb, h->precision == OCEAN_PREC_FP64, true, h->quad_tail != 0, &NT, &TC, &TQ);
    int bb, S, chunk;
    bwd_geometry(h, &bb, &S, &chunk);
    const int W = bwd_waves(h);
    dim3 grid((unsigned)(((long long)h->Nk * bb * S + 7) / 8 * 8));   // 8 XCDs, whole rounds
    const int slot = prof_begin(h, "proj_bwd");
    hipError_t e;
    if (h->precision == OCEAN_PREC_FP64)
        e = bwd_dispatch<double>(W, NT, TC, TQ, grid, h->stream, h->U64, h->ws.phi, h->ws.part, h->Nk,
                                 h->Nx, h->Nb, cols, col0, ncb, bb, S, chunk);
    else
        e = bwd_dispatch<float>(W, NT, TC, TQ, grid, h->stream, h->U32, h->ws.phi, h->ws.part, h->Nk,
                                h->Nx, h->Nb, cols, col0, ncb, bb, S, chunk);
    prof_end(h, slot);
    return e;
}

}  // namespace ocean
