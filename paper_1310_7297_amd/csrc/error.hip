// Approximation error of a colour map against the exact one (Sec. V-A) and
// the error bounds of the MBR and tangential approximations (Sec. IV-A).
#include <cmath>
#include <vector>

#include "vcm_internal.h"

namespace vcm {
namespace {

constexpr int kErrBlocks = 1024;

// Per-block float64 partial sums of (ce - ca), |ce - ca| and ce; the host adds
// the partials in a fixed order, so the result does not depend on timing.
__global__ __launch_bounds__(256) void k_map_error(const float *__restrict__ ce,
                                                   const float *__restrict__ ca, int64_t n,
                                                   double *__restrict__ part) {
    __shared__ double s[3][256];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * 256) {
        const double e = ce[i], x = ca[i];
        a += e - x;
        b += fabs(e - x);
        c += e;
    }
    s[0][threadIdx.x] = a;
    s[1][threadIdx.x] = b;
    s[2][threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < 3; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) part[3 * blockIdx.x + k] = s[k][0];
}

}  // namespace

vcm_status map_error(const float *ce, const float *ca, int64_t n, hipStream_t s, double *out) {
    out[0] = out[1] = 0.0;
    if (n <= 0) return VCM_OK;
    double *part = nullptr;
    hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&part), sizeof(double) * 3 * kErrBlocks, s);
    if (e != hipSuccess) return set_error(VCM_E_NOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    const int blocks = static_cast<int>(std::min<int64_t>(kErrBlocks, (n + 255) / 256));
    hipLaunchKernelGGL(k_map_error, dim3(blocks), dim3(256), 0, s, ce, ca, n, part);
    std::vector<double> h(3 * blocks);
    e = hipMemcpyAsync(h.data(), part, sizeof(double) * 3 * blocks, hipMemcpyDeviceToHost, s);
    hipFreeAsync(part, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_error(VCM_E_DEVICE, std::string("map error: ") + hipGetErrorString(e));
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = 0; i < blocks; ++i) {
        a += h[3 * i];
        b += h[3 * i + 1];
        c += h[3 * i + 2];
    }
    out[0] = c > 0 ? a / c : 0.0;
    out[1] = c > 0 ? b / c : 0.0;
    return VCM_OK;
}

// The bounds as printed: for each ring with radii r_i < r_{i+1}, n = (dr -
// r_{i+1}) / (r_{i+1} - r_i) rings can be mis-coloured, a_i bands lie below the
// stated angle, and every cell of the ring contributes n a_i mu times its
// size (area in the meridian quadrant in 2-D, volume of revolution about the
// normal in 3-D).  MBR: dr = sqrt(2) r_{i+1}, angle arctan(r_{i+1} / (S/2));
// tangent: dr = sqrt(r_{i+1}^2 + (r_{i+1} - r_i)^2), angle
// arctan(r_{i+1} / (S/2 + r_i)).
void error_bounds(double S, double mu, double d0, int dim, double *out) {
    double V0;
    const int K = count_rings(S, mu, d0, &V0);
    auto radius = [&](int i) -> double {
        if (i <= 0) return d0;
        if (i > K) return S / (2.0 * std::tan(mu / 2.0));
        return S / (2.0 * std::tan((V0 - i * mu) / 2.0));
    };
    double E[2] = {0.0, 0.0};
    std::vector<double> g;
    for (int i = 0; i <= K; ++i) {
        const double r0 = radius(i), r1 = radius(i + 1);
        if (!(r1 > r0)) continue;
        const double dp = 0.5 * (r0 + r1), W0 = 2.0 * std::atan(S / (2.0 * dp));
        g.clear();
        g.push_back(M_PI / 2.0);
        for (int j = 1;; ++j) {
            const double W = W0 - j * mu;
            if (W < mu) break;
            g.push_back((M_PI / 2.0) * (2.0 * dp * std::tan(W / 2.0)) / S);
        }
        g.push_back(0.0);
        const int L = static_cast<int>(g.size()) - 1;
        double size = 0.0;
        for (int j = 0; j < L; ++j) {
            if (dim == 2)
                size += 0.5 * (g[j] - g[j + 1]) * (r1 * r1 - r0 * r0);
            else
                size += 2.0 * M_PI * (r1 * r1 * r1 - r0 * r0 * r0) / 3.0 *
                        (std::sin(g[j]) - std::sin(g[j + 1]));
        }
        const double dr[2] = {std::sqrt(2.0) * r1, std::sqrt(r1 * r1 + (r1 - r0) * (r1 - r0))};
        const double lim[2] = {std::atan(r1 / (S / 2.0)), std::atan(r1 / (S / 2.0 + r0))};
        for (int m = 0; m < 2; ++m) {
            int a = 0;
            for (int j = 0; j < L; ++j)
                if (g[j + 1] < lim[m]) ++a;
            E[m] += (dr[m] - r1) / (r1 - r0) * a * mu * size;
        }
    }
    out[0] = E[0];
    out[1] = E[1];
}

}  // namespace vcm
