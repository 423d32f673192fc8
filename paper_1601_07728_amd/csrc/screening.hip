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
// One kernel computes, for a 64 x 64 tile pair (I <= J, the rest is the mirror) and one node, the
// two complex products on the FP64 matrix cores and folds |A|^2 - |B|^2 into a per-node partial;
// G is never written.  A second kernel adds the node partials in node order and mirrors the tiles.
#include <map>
#include <mutex>
#include <type_traits>

#include "internal.h"

namespace ocean {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;          // rows (and columns) of a tile pair
constexpr int kWaves = 4;          // wave w: rows 16 w .. 16 w + 15 of the I tile, all 64 columns
constexpr int kKS = 16;            // states per staged chunk
constexpr int kRP = kTile + 1;     // LDS pitch (double2) of a staged row-side state: odd, spreads banks
constexpr int kCP = kTile + 4;     // LDS pitch (double) of one part of a staged column-side state

// Block = (tile pair, node); blockIdx is renumbered so that the nodes of one tile pair run on one
// XCD (blocks are dealt round-robin over the 8 XCDs), where they share the tiles' rows in L2.
// A real GEMM over k = (state s, part p) whose rows are (r, q), q = 0 for the real and 1 for the
// imaginary part of the result, and whose columns are the points r':
//   X[(r, q)][(s, p)] = d_s * (q == 0 ? (Re, Im) psi_s(r) : (Im, -Re) psi_s(r))[p]
//   Y[(s, p)][r']     = (Re, Im) psi_s(r')[p]
// gives row (r, 0) = Re and row (r, 1) = Im of sum_s psi_s(r) conj(psi_s(r')) d_s for real d_s.
// The structure sits on the row side, which a lane reads once per k-step for all of its column
// tiles; the column side is a plain read of a planar (Re plane, Im plane) staged copy.
// One 16x16x4 MFMA k-step covers two states (lane l = i + 16 kq, kq = 2 (state) + part).
// Each wave holds 2 row tiles (16 complex rows) x 4 column tiles, for A and for B.
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(2))) void chi0_node_kernel(
    const double2* __restrict__ psi, const double* __restrict__ eps, int n_points, int n_states, double mu,
    const double* __restrict__ tnodes, const double* __restrict__ wnodes, int n_t, int n_tiles, int n_pairs,
    double* __restrict__ part) {
    __shared__ __align__(16) double2 sR[2][kKS][kRP];
    __shared__ __align__(16) double sC[2][kKS][2 * kCP + 1];
    __shared__ double2 sD[2][kKS];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
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

    // staging: element e of a chunk is psi[row][s0 + e % 16] for row e / 16 of the 128 rows (I's
    // 64, then J's 64): 16 lanes read one row's 256 contiguous bytes.  The loads of the next
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
            v[m] = psi[(size_t)min(rg, n_points - 1) * n_states + min(s, n_states - 1)];
        }
    };
    auto store = [&](int buf, int s0, const double2 (&v)[PRE]) {
#pragma unroll
        for (int m = 0; m < PRE; ++m) {
            const int e = threadIdx.x + 64 * kWaves * m;
            const int rl = e / kKS, sl = e - rl * kKS;
            if (rl < kTile) {
                sR[buf][sl][rl] = v[m];
            } else {
                sC[buf][sl][rl - kTile] = v[m].x;
                sC[buf][sl][kCP + rl - kTile] = v[m].y;
            }
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

    const int p = kq & 1;              // part of the k index this lane holds
    const int q = i & 1;               // re/im row of the A operand this lane holds
    const bool take_re = p == q;       // X[(r, q)][(s, p)] is +-Re psi when p == q, else Im psi
    const double sgn = (p & q) ? -1.0 : 1.0;
    // row tiles and column tiles that hold points (the last tile of the grid is ragged); the
    // counts are wave-uniform, so the guards below are scalar branches
    const int rows_left = n_points - (r0 + 16 * wave);
    const int n_rt = rows_left <= 0 ? 0 : (rows_left > 8 ? 2 : 1);
    const int n_ct = min(4, (n_points - c0 + 15) / 16);
    const bool full = n_rt == 2 && n_ct == 4;

    // the whole contraction and epilogue, instantiated twice so that the full tiles run without
    // guards and each instance gets its own register allocation
    auto run = [&](auto guard_tag) {
        constexpr bool guard = decltype(guard_tag)::value;
        v4d accA[2][4], accB[2][4];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) accA[rt][ct] = accB[rt][ct] = v4d{0, 0, 0, 0};
        auto kstep = [&](int buf, int ks) {
            const int sl = 2 * ks + (kq >> 1);
            const double2 d = sD[buf][sl];
            const double wa = sgn * d.x, wb = sgn * d.y;
            double ya[4];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) ya[ct] = sC[buf][sl][p * kCP + 16 * ct + i];
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                if (guard && rt >= n_rt) continue;
                const double2 x = sR[buf][sl][16 * wave + 8 * rt + (i >> 1)];
                const double v = take_re ? x.x : x.y;
                const double xa = v * wa, xb = v * wb;
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    if (guard && ct >= n_ct) continue;
                    accA[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, ya[ct], accA[rt][ct], 0, 0, 0);
                    accB[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(xb, ya[ct], accB[rt][ct], 0, 0, 0);
                }
            }
        };

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
            for (int ks = 0; ks < kKS / 2; ++ks) kstep(buf, ks);
            if (more) store(buf ^ 1, (ch + 1) * kKS, pre);
            __syncthreads();
        }

        // |A|^2 - |B|^2 of each complex element: lane (i, kq) register r of tile (rt, ct) holds real
        // row 4 r + kq of the row tile, i.e. point 8 rt + 2 r + kq / 2 of the wave's rows, part kq % 2,
        // and column 16 ct + i; the partner lane kq ^ 1 (lane ^ 16) holds the other part
        const double c = wnodes[node] * 0.31830988618379067154;   // w_j / pi
        double* out = part + (size_t)node * n_points * n_points;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double v = accA[rt][ct][r] * accA[rt][ct][r] - accB[rt][ct][r] * accB[rt][ct][r];
                    const double both = v + __shfl_xor(v, 16);
                    const int row = r0 + 16 * wave + 8 * rt + 2 * r + (kq >> 1);
                    const int col = c0 + 16 * ct + i;
                    if ((kq & 1) == 0 && row < n_points && col < n_points) out[(size_t)row * n_points + col] = c * both;
                }
    };
    if (full) run(std::false_type{});
    else run(std::true_type{});
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

// Device scratch of the response build (the node partials, then the energies, nodes and
// weights), kept per device between calls and grown on demand, so that repeated builds do not
// pay an allocation and a free each; ocean_screening_release gives it back.  The mutex also
// serialises the builds, which share it.
struct ScreeningScratch {
    void* ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_scratch_mu;
std::map<int, ScreeningScratch> g_scratch;   // by device

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
    int rc = OCEAN_OK;
    auto fail = [&](int code, const std::string& what) {
        (void)hipGetLastError();
        set_error("ocean_screening_chi0: " + what);
        rc = code;
    };
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) {
        fail(OCEAN_ERR_DEVICE, "hipGetDevice failed");
        return rc;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ScreeningScratch& ws = g_scratch[device];
    const size_t need = ((size_t)n2 * n_t + (size_t)n_states + 2 * (size_t)n_t) * sizeof(double);
    if (ws.bytes < need) {
        // the previous build on this device synchronised its stream before returning
        if (ws.ptr) (void)hipFree(ws.ptr);
        ws.ptr = nullptr;
        ws.bytes = 0;
        if (hipMalloc(&ws.ptr, need) != hipSuccess) {
            ws.ptr = nullptr;
            fail(OCEAN_ERR_OUT_OF_MEMORY, "hipMalloc failed");
            return rc;
        }
        ws.bytes = need;
    }
    double* part = static_cast<double*>(ws.ptr);   // [n_t][n_points][n_points]
    double* dev = part + (size_t)n2 * n_t;         // eps [n_states], t [n_t], w [n_t]
    double* eps_dev = dev;
    double* t_dev = dev + n_states;
    double* w_dev = t_dev + n_t;
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
    return rc;
}

extern "C" int ocean_screening_release(void) {
    set_error("");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    int current = 0;
    const bool have_current = hipGetDevice(&current) == hipSuccess;
    int rc = OCEAN_OK;
    for (auto& kv : g_scratch) {
        if (!kv.second.ptr) continue;
        if (hipSetDevice(kv.first) != hipSuccess || hipFree(kv.second.ptr) != hipSuccess) {
            (void)hipGetLastError();
            set_error("ocean_screening_release: hipFree failed");
            rc = OCEAN_ERR_DEVICE;
        }
    }
    g_scratch.clear();
    if (have_current) (void)hipSetDevice(current);
    return rc;
}
