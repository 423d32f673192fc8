// Static RPA response of the screening stage (section 3.3, eq. chi_rpa at omega = 0, with the
// Green's function of eq. greens.fcn on the real-space grid around the core site):
//
//   G_j(r, r') = sum_s psi_s(r) psi_s*(r') d_j(s),   d_j(s) = 1 / (mu + i t_j - eps_s)
//   chi0(r, r') = sum_j (w_j / pi) Re[G_j(r, r') G_j(r', r)]
//
// The frequency integral runs along the imaginary axis through mu; the integrand at -t is the
// complex conjugate of the one at t, so only t >= 0 is summed, with caller-given nodes t_j and
// weights w_j.
//
// Splitting d_j into its real and imaginary parts gives two Hermitian matrices,
//   A_j = Psi diag(Re d_j) Psi^H,  B_j = Psi diag(Im d_j) Psi^H,  G_j = A_j + i B_j,
// and G_j(r', r) = conj(A_j(r, r')) + i conj(B_j(r, r')), so that
//   Re[G_j(r, r') G_j(r', r)] = |A_j(r, r')|^2 - |B_j(r, r')|^2.
// One kernel computes, for a 48 x 48 tile pair (I <= J, the rest is the mirror) and one node, the
// two complex products on the FP64 matrix cores and folds |A|^2 - |B|^2 into a per-node partial;
// G is never written.  A second kernel adds the node partials in node order and mirrors the tiles.
#include "internal.h"

namespace ocean {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kTile = 48;          // rows (and complex columns) of a tile pair
constexpr int kWaves = kTile / 16; // one wave per 16 rows, all 48 complex columns
constexpr int kCT = 2 * kTile / 16;  // real column tiles of 16: (column, re/im) interleaved
constexpr int kKS = 16;            // states per staged chunk
constexpr int kRP = kTile + 1;     // LDS row pitch (complex) of a staged state: odd, spreads banks

// Block = (tile pair, node); blockIdx is renumbered so that the nodes of one tile pair run on one
// XCD (blocks are dealt round-robin over the 8 XCDs), where they share the tiles' rows in L2.
// Wave w: rows I + 16 w .. +15; lane l = i + 16 kq.  A real GEMM over k = (state s, part p):
//   X[r][(s, p)] = (Re, Im) psi_s(r);  Y[(s, p)][(r', q)] = d_s M_pq(psi_s(r')) with
//   M = [[Re, -Im], [Im, Re]] gives (Re, Im) of sum_s psi_s(r) conj(psi_s(r')) d_s for real d_s.
// One 16x16x4 MFMA k-step covers two states (kq = 2 (state) + part).
__global__ __launch_bounds__(64 * kWaves) void chi0_node_kernel(
    const double2* __restrict__ psi, const double* __restrict__ eps, int n_points, int n_states, double mu,
    const double* __restrict__ tnodes, const double* __restrict__ wnodes, int n_t, int n_tiles, int n_pairs,
    double* __restrict__ part) {
    __shared__ __align__(16) double2 sR[2][kKS][kRP];
    __shared__ __align__(16) double2 sC[2][kKS][kRP];
    __shared__ double2 sD[2][kKS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    // XCD-aware numbering: block b runs on XCD b % 8; give each XCD a contiguous run of
    // (pair, node) items, node fastest
    const int total = n_pairs * n_t;
    const int per_xcd = (total + 7) / 8;
    const int item = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (item >= total) return;
    const int node = item % n_t;
    int pr = item / n_t;
    // pair index -> (I, J), I <= J, row-major over the upper triangle
    int I = 0;
    while (pr >= n_tiles - I) {
        pr -= n_tiles - I;
        ++I;
    }
    const int J = I + pr;
    const int r0 = I * kTile, c0 = J * kTile;
    const double tj = tnodes[node];

    // staging: element e of a chunk is psi[row][s0 + e % 16] for row e / 16 of the 96 rows (I's
    // 48, then J's 48): 16 lanes read one row's 256 contiguous bytes.  The loads of the next
    // chunk are issued before the current chunk's MFMAs and written to LDS after them.
    constexpr int PRE = 2 * kTile * kKS / (64 * kWaves);
    static_assert(PRE * 64 * kWaves == 2 * kTile * kKS, "staging split");
    auto load = [&](int s0, double2 (&v)[PRE]) {
#pragma unroll
        for (int m = 0; m < PRE; ++m) {
            const int e = threadIdx.x + 64 * kWaves * m;
            const int rl = e / kKS, sl = e - rl * kKS;
            const int rg = rl < kTile ? r0 + rl : c0 + rl - kTile;
            const int s = s0 + sl;
            v[m] = (rg < n_points && s < n_states) ? psi[(size_t)rg * n_states + s] : make_double2(0.0, 0.0);
        }
    };
    auto store = [&](int buf, int s0, const double2 (&v)[PRE]) {
#pragma unroll
        for (int m = 0; m < PRE; ++m) {
            const int e = threadIdx.x + 64 * kWaves * m;
            const int rl = e / kKS, sl = e - rl * kKS;
            if (rl < kTile) sR[buf][sl][rl] = v[m];
            else sC[buf][sl][rl - kTile] = v[m];
        }
        if (threadIdx.x < kKS) {
            const int s = s0 + threadIdx.x;
            double2 d = make_double2(0.0, 0.0);
            if (s < n_states) {
                // 1 / (a + i t) = (a - i t) / (a^2 + t^2), a = mu - eps_s
                const double a = mu - eps[s];
                const double den = a * a + tj * tj;
                d = make_double2(a / den, -tj / den);
            }
            sD[buf][threadIdx.x] = d;
        }
    };

    v4d accA[kCT], accB[kCT];
#pragma unroll
    for (int t = 0; t < kCT; ++t) accA[t] = accB[t] = v4d{0, 0, 0, 0};
    const int p = kq & 1;              // part of the k index this lane holds
    const int q = i & 1;               // re/im of the output column this lane holds (B operand)
    const int rloc = wave * 16 + i;    // A operand row within the tile
    // M_pq: the component of psi_s(r') and its sign
    const bool take_re = p == q;
    const double sgn = (p == 0 && q == 1) ? -1.0 : 1.0;

    const int n_chunks = (n_states + kKS - 1) / kKS;
    double2 pre[PRE];
    load(0, pre);
    store(0, 0, pre);
    __syncthreads();
    for (int ch = 0; ch < n_chunks; ++ch) {
        const int buf = ch & 1;
        const bool more = ch + 1 < n_chunks;
        if (more) load((ch + 1) * kKS, pre);
#pragma unroll
        for (int ks = 0; ks < kKS / 2; ++ks) {
            const int sl = 2 * ks + (kq >> 1);
            const double2 x = sR[buf][sl][rloc];
            const double a = p ? x.y : x.x;
            const double2 d = sD[buf][sl];
            const double wa = sgn * d.x, wb = sgn * d.y;
#pragma unroll
            for (int t = 0; t < kCT; ++t) {
                const double2 y = sC[buf][sl][8 * t + (i >> 1)];
                const double m = take_re ? y.x : y.y;
                accA[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, wa * m, accA[t], 0, 0, 0);
                accB[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, wb * m, accB[t], 0, 0, 0);
            }
        }
        if (more) store(buf ^ 1, (ch + 1) * kKS, pre);
        __syncthreads();
    }

    // |A|^2 - |B|^2 of each complex element: lane (i, kq) register r holds row 4 r + kq and real
    // column 16 t + i = (column 8 t + i / 2, re/im i % 2); the partner lane i ^ 1 holds the other part
    const double c = wnodes[node] * 0.31830988618379067154;   // w_j / pi
    double* out = part + (size_t)node * n_points * n_points;
#pragma unroll
    for (int t = 0; t < kCT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double v = accA[t][r] * accA[t][r] - accB[t][r] * accB[t][r];
            const double both = v + __shfl_xor(v, 1);
            const int row = r0 + wave * 16 + 4 * r + kq;
            const int col = c0 + 8 * t + (i >> 1);
            if (q == 0 && row < n_points && col < n_points) out[(size_t)row * n_points + col] = c * both;
        }
}

// chi0[r][r'] = sum over nodes of the partials, in node order; each element reads the upper
// triangle tile that holds it (the partials of the tiles below the diagonal are mirrored)
__global__ __launch_bounds__(256) void chi0_sum_kernel(const double* __restrict__ part, int n_points, int n_t,
                                                       double* __restrict__ chi0) {
    const long long n2 = (long long)n_points * n_points;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n2;
         e += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(e / n_points), c = (int)(e - (long long)r * n_points);
        // the element lives in the computed tile pair (min tile, max tile)
        const bool upper = r / kTile <= c / kTile;
        const size_t src = upper ? (size_t)e : (size_t)c * n_points + r;
        double s = 0.0;
        for (int j = 0; j < n_t; ++j) s += part[(size_t)j * n2 + src];
        chi0[e] = s;
    }
}

}  // namespace
}  // namespace ocean

using namespace ocean;

extern "C" int ocean_screening_chi0(const double* psi_dev, const double* eps, int n_points, int n_states,
                                    double mu, const double* t, const double* w, int n_t, double* chi0_dev,
                                    void* stream) {
    set_error("");
    if (!psi_dev || !eps || !t || !w || !chi0_dev || n_points < 1 || n_states < 1 || n_t < 1 ||
        !std::isfinite(mu)) {
        set_error("ocean_screening_chi0: invalid argument");
        return OCEAN_ERR_INVALID_ARG;
    }
    for (int s = 0; s < n_states; ++s)
        if (!std::isfinite(eps[s])) {
            set_error("ocean_screening_chi0: energies must be finite");
            return OCEAN_ERR_INVALID_ARG;
        }
    for (int j = 0; j < n_t; ++j)
        if (!std::isfinite(t[j]) || !std::isfinite(w[j]) || t[j] < 0.0) {
            set_error("ocean_screening_chi0: nodes must be finite and >= 0, weights finite");
            return OCEAN_ERR_INVALID_ARG;
        }
    const long long n2 = (long long)n_points * n_points;
    if ((long long)n_points * n_states >= (1LL << 40) || n2 * n_t >= (1LL << 40)) {
        set_error("ocean_screening_chi0: problem too large");
        return OCEAN_ERR_INVALID_ARG;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* part = nullptr;
    double* dev = nullptr;   // eps [n_states], t [n_t], w [n_t]
    int rc = OCEAN_OK;
    auto fail = [&](int code, const std::string& what) {
        (void)hipGetLastError();
        set_error("ocean_screening_chi0: " + what);
        rc = code;
    };
    if (hipMalloc((void**)&part, (size_t)n2 * n_t * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&dev, ((size_t)n_states + 2 * (size_t)n_t) * sizeof(double)) != hipSuccess)
        fail(OCEAN_ERR_OUT_OF_MEMORY, "hipMalloc failed");
    double* eps_dev = dev;
    double* t_dev = dev ? dev + n_states : nullptr;
    double* w_dev = dev ? t_dev + n_t : nullptr;
    if (rc == OCEAN_OK &&
        (hipMemcpyAsync(eps_dev, eps, (size_t)n_states * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
         hipMemcpyAsync(t_dev, t, (size_t)n_t * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
         hipMemcpyAsync(w_dev, w, (size_t)n_t * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess))
        fail(OCEAN_ERR_DEVICE, "upload failed");
    const int n_tiles = (n_points + kTile - 1) / kTile;
    const int n_pairs = n_tiles * (n_tiles + 1) / 2;
    const long long items = (long long)n_pairs * n_t;
    if (rc == OCEAN_OK) {
        const unsigned blocks = (unsigned)((items + 7) / 8 * 8);
        chi0_node_kernel<<<blocks, 64 * kWaves, 0, st>>>(reinterpret_cast<const double2*>(psi_dev), eps_dev, n_points,
                                                        n_states, mu, t_dev, w_dev, n_t, n_tiles, n_pairs, part);
        if (hipGetLastError() != hipSuccess) fail(OCEAN_ERR_DEVICE, "chi0 launch");
    }
    if (rc == OCEAN_OK) {
        const unsigned blocks = (unsigned)std::min<long long>((n2 + 255) / 256, 8192);
        chi0_sum_kernel<<<blocks, 256, 0, st>>>(part, n_points, n_t, chi0_dev);
        if (hipGetLastError() != hipSuccess) fail(OCEAN_ERR_DEVICE, "sum launch");
    }
    if (rc == OCEAN_OK && hipStreamSynchronize(st) != hipSuccess) fail(OCEAN_ERR_DEVICE, "synchronize");
    if (part) (void)hipFree(part);
    if (dev) (void)hipFree(dev);
    return rc;
}
