// Static RPA response of the screening stage (section 3.3, eq. chi_rpa at omega = 0, with the
// Green's function of eq. greens.fcn on the real-space grid around the core site):
//
//   G_j(r, r') = sum_s psi_s(r) psi_s*(r') / (mu + i t_j - eps_s)
//   chi0(r, r') = sum_j (w_j / pi) Re[G_j(r, r') G_j(r', r)]
//
// The frequency integral runs along the imaginary axis through mu; the integrand at -t is the
// complex conjugate of the one at t, so only t >= 0 is summed, with caller-given nodes t_j and
// weights w_j.  Per node, one kernel scales the state columns of psi by 1/(mu + i t_j - eps_s),
// one complex GEMM on the matrix cores forms G_j (rocBLAS: a plain GEMM), and one kernel adds
// the symmetric product into chi0.
#include <rocblas/rocblas.h>

#include "internal.h"

namespace ocean {
namespace {

// y[r][s] = psi[r][s] / (mu + i t - eps[s]), row-major [n_points][n_states]
__global__ __launch_bounds__(256) void scale_states_kernel(const double2* __restrict__ psi,
                                                           const double* __restrict__ eps, double mu,
                                                           double t, double2* __restrict__ y,
                                                           long long n_points, int n_states) {
    const long long total = n_points * n_states;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int s = (int)(e % n_states);
        // 1 / (a + i t) = (a - i t) / (a^2 + t^2), a = mu - eps
        const double a = mu - eps[s];
        const double d = a * a + t * t;
        const double gr = a / d, gi = -t / d;
        const double2 p = psi[e];
        y[e] = make_double2(p.x * gr - p.y * gi, p.x * gi + p.y * gr);
    }
}

// chi0[r][r'] += c Re(G[r][r'] G[r'][r]) over 32 x 32 tiles: the tile and its mirror are
// staged in LDS so that both reads coalesce.
__global__ __launch_bounds__(256) void accumulate_chi0_kernel(const double2* __restrict__ g,
                                                              double* __restrict__ chi0, int n,
                                                              double c) {
    __shared__ double2 mir[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    // mirror tile: G[c0 + i][r0 + j] -> mir[j][i]
    for (int i = ty; i < 32; i += 8) {
        const int row = c0 + i, col = r0 + tx;
        mir[tx][i] = (row < n && col < n) ? g[(size_t)row * n + col] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const int row = r0 + i, col = c0 + tx;
        if (row < n && col < n) {
            const double2 a = g[(size_t)row * n + col];
            const double2 b = mir[i][tx];
            chi0[(size_t)row * n + col] += c * (a.x * b.x - a.y * b.y);
        }
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
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t ny = (size_t)n_points * n_states, ng = (size_t)n_points * n_points;
    double2* y = nullptr;
    double2* g = nullptr;
    double* eps_dev = nullptr;
    rocblas_handle blas = nullptr;
    int rc = OCEAN_OK;
    auto fail = [&](int code, const std::string& what) {
        (void)hipGetLastError();
        set_error("ocean_screening_chi0: " + what);
        rc = code;
    };
    if (hipMalloc((void**)&y, ny * sizeof(double2)) != hipSuccess ||
        hipMalloc((void**)&g, ng * sizeof(double2)) != hipSuccess ||
        hipMalloc((void**)&eps_dev, (size_t)n_states * sizeof(double)) != hipSuccess)
        fail(OCEAN_ERR_OUT_OF_MEMORY, "hipMalloc failed");
    if (rc == OCEAN_OK && hipMemcpyAsync(eps_dev, eps, (size_t)n_states * sizeof(double), hipMemcpyHostToDevice,
                                         st) != hipSuccess)
        fail(OCEAN_ERR_DEVICE, "energy upload failed");
    if (rc == OCEAN_OK && hipMemsetAsync(chi0_dev, 0, ng * sizeof(double), st) != hipSuccess)
        fail(OCEAN_ERR_DEVICE, "clearing chi0 failed");
    if (rc == OCEAN_OK && (rocblas_create_handle(&blas) != rocblas_status_success ||
                           rocblas_set_stream(blas, st) != rocblas_status_success))
        fail(OCEAN_ERR_DEVICE, "rocBLAS handle");
    const double2* psi = reinterpret_cast<const double2*>(psi_dev);
    const unsigned sblocks = (unsigned)std::min<size_t>((ny + 255) / 256, 8192);
    const dim3 tgrid((unsigned)((n_points + 31) / 32), (unsigned)((n_points + 31) / 32));
    for (int j = 0; j < n_t && rc == OCEAN_OK; ++j) {
        scale_states_kernel<<<sblocks, 256, 0, st>>>(psi, eps_dev, mu, t[j], y, n_points, n_states);
        if (hipGetLastError() != hipSuccess) {
            fail(OCEAN_ERR_DEVICE, "scale launch");
            break;
        }
        // column-major view: X = psi^T (n_states x n_points, ld n_states), Y likewise;
        // C = X^H Y is n_points x n_points with C(r', r) = G(r, r'), i.e. G row-major
        const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
        if (rocblas_zgemm(blas, rocblas_operation_conjugate_transpose, rocblas_operation_none, n_points, n_points,
                          n_states, &one, reinterpret_cast<const rocblas_double_complex*>(psi), n_states,
                          reinterpret_cast<const rocblas_double_complex*>(y), n_states, &zero,
                          reinterpret_cast<rocblas_double_complex*>(g), n_points) != rocblas_status_success) {
            fail(OCEAN_ERR_DEVICE, "rocblas_zgemm failed");
            break;
        }
        accumulate_chi0_kernel<<<tgrid, 256, 0, st>>>(g, chi0_dev, n_points, w[j] / M_PI);
        if (hipGetLastError() != hipSuccess) fail(OCEAN_ERR_DEVICE, "accumulate launch");
    }
    if (rc == OCEAN_OK && hipStreamSynchronize(st) != hipSuccess) fail(OCEAN_ERR_DEVICE, "synchronize");
    if (blas) (void)rocblas_destroy_handle(blas);
    if (y) (void)hipFree(y);
    if (g) (void)hipFree(g);
    if (eps_dev) (void)hipFree(eps_dev);
    return rc;
}
