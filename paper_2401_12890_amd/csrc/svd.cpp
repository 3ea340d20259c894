// Thin SVD of the dictionary in float64 by one-sided (Hestenes) Jacobi.
//
// Algorithm 2 of the paper starts from the SVD of K (Sec. III-E); the
// truncated factors give the low-rank inverse of Eq. (DictVecSVD). One-sided
// Jacobi orthogonalises the min(P, Q) rows (or columns) of K directly, so the
// small singular values and their vectors keep high relative accuracy; a
// Gram-matrix eigensolve would square the condition number. Pairs are
// visited in round-robin (tournament) order so the n/2 rotations of a round
// touch disjoint rows and run on host threads in parallel.
#include "internal.h"

#include <algorithm>
#include <atomic>
#include <barrier>
#include <cmath>
#include <numeric>
#include <thread>
#include <vector>

namespace ssmap {

namespace {

// A holds n vectors of length L (row-major n x L). Gt (n x n, row-major)
// accumulates the rotations transposed: on exit A = Gt A0 with mutually
// orthogonal rows, i.e. A0 = Gt^T A.
void jacobi_rows(std::vector<double> &A, int n, int L, std::vector<double> &G) {
    G.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) G[(size_t)i * n + i] = 1.0;
    if (n < 2) return;
    const int m = (n % 2) ? n + 1 : n;          // players, one bye if n is odd
    // pairs count as orthogonal once |a_i . a_j| <= sqrt(L) eps ||a_i|| ||a_j||;
    // rows whose norm is at the rounding level of ||A||_F (below 4 eps ||A||_F)
    // are numerically zero and are left alone
    const double eps = 2.220446049250313e-16;
    const double tol = std::sqrt((double)L) * eps;
    double fro2 = 0.0;
    for (double v : A) fro2 += v * v;
    const double negligible2 = fro2 * (4 * eps) * (4 * eps);
    unsigned hw = std::thread::hardware_concurrency();
    int nthreads = (int)std::min<unsigned>(hw ? hw : 1, 16);
    const double work = (double)n * n * L;
    if (work < 4e6) nthreads = 1;
    nthreads = std::max(1, std::min(nthreads, m / 2));

    std::vector<int> ring(m);
    std::iota(ring.begin(), ring.end(), 0);
    std::atomic<int> rotated{0};
    std::atomic<bool> done{false};
    int sweep = 0;
    const int max_sweeps = 60;

    auto rotate_pair = [&](int i, int j) -> bool {
        if (i >= n || j >= n) return false;
        double *ai = &A[(size_t)i * L], *aj = &A[(size_t)j * L];
        double alpha = 0.0, beta = 0.0, gamma = 0.0;
        for (int k = 0; k < L; ++k) {
            alpha += ai[k] * ai[k];
            beta += aj[k] * aj[k];
            gamma += ai[k] * aj[k];
        }
        if (alpha <= negligible2 || beta <= negligible2) return false;
        if (gamma == 0.0 || !(std::fabs(gamma) > tol * std::sqrt(alpha * beta))) return false;
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t);
        const double s = c * t;
        for (int k = 0; k < L; ++k) {
            const double x = ai[k], y = aj[k];
            ai[k] = c * x - s * y;
            aj[k] = s * x + c * y;
        }
        double *gi = &G[(size_t)i * n], *gj = &G[(size_t)j * n];   // rows i, j of Gt
        for (int k = 0; k < n; ++k) {
            const double x = gi[k], y = gj[k];
            gi[k] = c * x - s * y;
            gj[k] = s * x + c * y;
        }
        return true;
    };

    // Round-robin schedule: player ring[0] is fixed, the others rotate.
    auto pair_of = [&](int round, int slot, int &a, int &b) {
        // positions in the rotated ring for this round
        auto pos = [&](int p) -> int {
            if (p == 0) return 0;
            return 1 + ((p - 1 + round) % (m - 1));
        };
        a = pos(slot);
        b = pos(m - 1 - slot);
        if (a > b) std::swap(a, b);
    };

    if (nthreads == 1) {
        for (sweep = 0; sweep < max_sweeps; ++sweep) {
            int cnt = 0;
            for (int round = 0; round < m - 1; ++round)
                for (int slot = 0; slot < m / 2; ++slot) {
                    int a, b;
                    pair_of(round, slot, a, b);
                    cnt += rotate_pair(a, b);
                }
            if (cnt == 0) break;
        }
        return;
    }

    std::barrier sync(nthreads);
    auto worker = [&](int tid) {
        for (int sw = 0; sw < max_sweeps; ++sw) {
            for (int round = 0; round < m - 1; ++round) {
                int local = 0;
                for (int slot = tid; slot < m / 2; slot += nthreads) {
                    int a, b;
                    pair_of(round, slot, a, b);
                    local += rotate_pair(a, b);
                }
                if (local) rotated.fetch_add(local, std::memory_order_relaxed);
                sync.arrive_and_wait();
            }
            // every thread reads the sweep's count, then thread 0 resets it
            const bool finished = rotated.load() == 0;
            sync.arrive_and_wait();
            if (tid == 0) rotated.store(0);
            sync.arrive_and_wait();
            if (finished) return;
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nthreads; ++t) pool.emplace_back(worker, t);
    worker(0);
    for (auto &th : pool) th.join();
    (void)done;
}

}  // namespace

// K is P x Q row-major. Outputs (k = min(P, Q)):
//   U (P x k row-major), s (k, descending), V (Q x k row-major),
// with K = U diag(s) V^T.
void thin_svd(const double *K, int P, int Q, std::vector<double> &U,
              std::vector<double> &s, std::vector<double> &V) {
    const bool rows = P <= Q;                   // orthogonalise the shorter side
    const int n = rows ? P : Q;
    const int L = rows ? Q : P;
    std::vector<double> A((size_t)n * L);
    if (rows) {
        std::copy(K, K + (size_t)P * Q, A.begin());
    } else {
        for (int p = 0; p < P; ++p)
            for (int q = 0; q < Q; ++q) A[(size_t)q * P + p] = K[(size_t)p * Q + q];
    }
    std::vector<double> G;
    jacobi_rows(A, n, L, G);
    std::vector<double> norm(n);
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int k = 0; k < L; ++k) acc += A[(size_t)i * L + k] * A[(size_t)i * L + k];
        norm[i] = std::sqrt(acc);
    }
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return norm[a] > norm[b]; });
    s.assign(n, 0.0);
    U.assign((size_t)P * n, 0.0);
    V.assign((size_t)Q * n, 0.0);
    for (int c = 0; c < n; ++c) {
        const int i = order[c];
        s[c] = norm[i];
        const double inv = norm[i] > 0 ? 1.0 / norm[i] : 0.0;
        // normalised orthogonal vector (length L) and the rotation column (length n)
        if (rows) {
            for (int q = 0; q < Q; ++q) V[(size_t)q * n + c] = A[(size_t)i * L + q] * inv;
            for (int p = 0; p < P; ++p) U[(size_t)p * n + c] = G[(size_t)i * n + p];
        } else {
            for (int p = 0; p < P; ++p) U[(size_t)p * n + c] = A[(size_t)i * L + p] * inv;
            for (int q = 0; q < Q; ++q) V[(size_t)q * n + c] = G[(size_t)i * n + q];
        }
    }
}

}  // namespace ssmap
