// Masked voxel sets (Sec. II-C, maskless footnote): only voxels inside the
// object are estimated, and the regulariser of Eq. (l2) runs over face-
// neighbour pairs whose two voxels are both inside. Host-side pieces:
//   * the per-voxel code byte the kernels read (bit 7: inside; bits 0..2:
//     number of inside face neighbours, 0..6),
//   * ||D^T D||_2 of the induced graph (twice the largest Laplacian
//     eigenvalue) by Lanczos in float64, for the xi_p rule of Eq. (sigma_cond),
//   * which bricks hold an inside voxel (bricks without one are not launched).
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace ssmap {

namespace {

// y = L x on the inside voxels (x, y indexed by voxel; outside entries stay 0).
void laplacian_apply(const Grid &g, const std::vector<uint8_t> &code, const std::vector<double> &x,
                     std::vector<double> &y) {
    const int64_t nx = g.nx, ny = g.ny, nz = g.nz, sy = nx, sz = nx * ny;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t yy = 0; yy < ny; ++yy)
            for (int64_t x0 = 0; x0 < nx; ++x0) {
                const int64_t n = x0 + nx * (yy + ny * z);
                if (!(code[n] & 0x80)) {
                    y[n] = 0.0;
                    continue;
                }
                double s = (double)(code[n] & 7) * x[n];
                // outside neighbours carry x = 0, so all box neighbours can be summed
                if (x0 > 0) s -= x[n - 1];
                if (x0 + 1 < nx) s -= x[n + 1];
                if (yy > 0) s -= x[n - sy];
                if (yy + 1 < ny) s -= x[n + sy];
                if (z > 0) s -= x[n - sz];
                if (z + 1 < nz) s -= x[n + sz];
                y[n] = s;
            }
}

// Largest eigenvalue of the symmetric tridiagonal (alpha, beta) by bisection
// on the Sturm sequence count.
double tridiag_max_eig(const std::vector<double> &al, const std::vector<double> &be) {
    const size_t k = al.size();
    double lo = 1e300, hi = -1e300;
    for (size_t i = 0; i < k; ++i) {               // Gershgorin interval
        const double r = (i > 0 ? std::fabs(be[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(be[i]) : 0.0);
        lo = std::min(lo, al[i] - r);
        hi = std::max(hi, al[i] + r);
    }
    auto count_above = [&](double x) {             // eigenvalues > x
        int neg = 0;
        double d = 1.0;
        for (size_t i = 0; i < k; ++i) {
            d = al[i] - x - (i > 0 ? be[i - 1] * be[i - 1] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            neg += d < 0.0;
        }
        return (int)k - neg;
    };
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (count_above(mid) >= 1) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

}  // namespace

void mask_codes(const Grid &g, const uint8_t *mask, std::vector<uint8_t> &code, int64_t &inside) {
    const int64_t nx = g.nx, ny = g.ny, nz = g.nz, N = g.N, sy = nx, sz = nx * ny;
    code.assign((size_t)N, 0);
    inside = 0;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t n = x + nx * (y + ny * z);
                if (!mask[n]) continue;
                int d = 0;
                d += x > 0 && mask[n - 1];
                d += x + 1 < nx && mask[n + 1];
                d += y > 0 && mask[n - sy];
                d += y + 1 < ny && mask[n + sy];
                d += z > 0 && mask[n - sz];
                d += z + 1 < nz && mask[n + sz];
                code[n] = (uint8_t)(0x80 | d);
                ++inside;
            }
}

double masked_dtd_norm(const Grid &g, const std::vector<uint8_t> &code) {
    const size_t N = (size_t)g.N;
    std::vector<double> v(N, 0.0), vprev(N, 0.0), w(N, 0.0);
    // start: the checkerboard on inside voxels (close to the top eigenvector
    // of grid graphs), slightly perturbed so no component is missing
    double nrm = 0.0;
    for (size_t n = 0; n < N; ++n)
        if (code[n] & 0x80) {
            const int64_t x = (int64_t)n % g.nx, y = ((int64_t)n / g.nx) % g.ny, z = (int64_t)n / (g.nx * g.ny);
            v[n] = ((x + y + z) & 1 ? -1.0 : 1.0) * (1.0 + 1e-3 * std::sin(0.37 * (double)n));
            nrm += v[n] * v[n];
        }
    if (nrm == 0.0) return 0.0;
    nrm = std::sqrt(nrm);
    for (double &e : v) e /= nrm;
    std::vector<double> al, be;
    double b_prev = 0.0, theta_prev = -1.0, theta = 0.0;
    int stable = 0;
    for (int k = 0; k < 400; ++k) {
        laplacian_apply(g, code, v, w);
        double a = 0.0;
        for (size_t n = 0; n < N; ++n) a += w[n] * v[n];
        double b = 0.0;
        for (size_t n = 0; n < N; ++n) {
            w[n] -= a * v[n] + b_prev * vprev[n];
            b += w[n] * w[n];
        }
        b = std::sqrt(b);
        al.push_back(a);
        theta = tridiag_max_eig(al, be);
        if (std::fabs(theta - theta_prev) <= 1e-15 * theta) {
            if (++stable >= 5) break;
        } else {
            stable = 0;
        }
        theta_prev = theta;
        if (b <= 1e-14 * std::max(1.0, theta)) break;   // invariant subspace found
        be.push_back(b);
        vprev.swap(v);
        for (size_t n = 0; n < N; ++n) v[n] = w[n] / b;
        b_prev = b;
    }
    return 2.0 * theta;                  // D^T D = 2 L
}

bool brick_has_inside(const Grid &g, const std::vector<uint8_t> &code, int64_t x0, int64_t y0,
                      int64_t z0, int tx, int ty, int tz) {
    for (int64_t z = z0; z < std::min<int64_t>(z0 + tz, g.nz); ++z)
        for (int64_t y = y0; y < std::min<int64_t>(y0 + ty, g.ny); ++y)
            for (int64_t x = x0; x < std::min<int64_t>(x0 + tx, g.nx); ++x)
                if (code[(size_t)(x + g.nx * (y + g.ny * z))] & 0x80) return true;
    return false;
}

}  // namespace ssmap
