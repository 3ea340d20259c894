// Host-only check of the library's CPU code, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitize.py (g++, no device
// code): the threaded one-sided Jacobi SVD, the mask codes and the Lanczos
// norm of a masked grid, the brick occupancy test, and the serving loop's
// first-fit allocator under random allocation and release. Exits non-zero on a
// failed check; the sanitizers abort on a memory or undefined-behaviour error.
#include "internal.h"
#include "slab.h"

#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

using namespace ssmap;

static int failures = 0;
#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++failures;                                                      \
        }                                                                    \
    } while (0)

// K = U diag(s) V^T within a relative tolerance, U and V with orthonormal columns.
static void check_svd(int P, int Q, unsigned seed, int rank_deficit) {
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd;
    std::vector<double> K((size_t)P * Q);
    for (auto &v : K) v = nd(rng);
    if (rank_deficit > 0 && P > 1)        // make the last rows copies of the first
        for (int p = P - rank_deficit; p < P; ++p)
            for (int q = 0; q < Q; ++q) K[(size_t)p * Q + q] = K[(size_t)(p % (P - rank_deficit)) * Q + q];
    std::vector<double> U, s, V;
    thin_svd(K.data(), P, Q, U, s, V);
    const int k = P < Q ? P : Q;
    CHECK((int)s.size() == k && U.size() == (size_t)P * k && V.size() == (size_t)Q * k);
    double fro = 0, err = 0;
    for (int p = 0; p < P; ++p)
        for (int q = 0; q < Q; ++q) {
            double v = 0;
            for (int i = 0; i < k; ++i) v += U[(size_t)p * k + i] * s[i] * V[(size_t)q * k + i];
            err += (v - K[(size_t)p * Q + q]) * (v - K[(size_t)p * Q + q]);
            fro += K[(size_t)p * Q + q] * K[(size_t)p * Q + q];
        }
    CHECK(std::sqrt(err) <= 1e-12 * std::sqrt(fro));
    for (int i = 1; i < k; ++i) CHECK(s[i] <= s[i - 1] && s[i] >= 0);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            double dv = 0;
            for (int q = 0; q < Q; ++q) dv += V[(size_t)q * k + i] * V[(size_t)q * k + j];
            if (s[i] > 1e-10 * s[0] && s[j] > 1e-10 * s[0]) CHECK(std::fabs(dv - (i == j)) <= 1e-10);
        }
}

static void check_masks(int64_t nx, int64_t ny, int64_t nz, double frac, unsigned seed) {
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> ud;
    const Grid g{nx, ny, nz, nx * ny * nz};
    std::vector<uint8_t> mask((size_t)g.N);
    for (auto &m : mask) m = ud(rng) < frac;
    std::vector<uint8_t> code;
    int64_t inside = 0;
    mask_codes(g, mask.data(), code, inside);
    CHECK((int64_t)code.size() == g.N);
    int64_t count = 0;
    for (int64_t n = 0; n < g.N; ++n) {
        count += mask[n] != 0;
        CHECK(((code[n] & 0x80u) != 0) == (mask[n] != 0));
        // bits 0..2: the number of inside face neighbours
        const int64_t x = n % nx, y = (n / nx) % ny, z = n / (nx * ny);
        int deg = 0;
        if (x > 0) deg += mask[n - 1] != 0;
        if (x + 1 < nx) deg += mask[n + 1] != 0;
        if (y > 0) deg += mask[n - nx] != 0;
        if (y + 1 < ny) deg += mask[n + nx] != 0;
        if (z > 0) deg += mask[n - nx * ny] != 0;
        if (z + 1 < nz) deg += mask[n + nx * ny] != 0;
        if (mask[n]) CHECK((int)(code[n] & 7u) == deg);
    }
    CHECK(count == inside);
    const double nrm = masked_dtd_norm(g, code);
    // ||D^T D|| = 2 lambda_max(L) of the inside graph lies in [0, 4 * max degree]
    CHECK(nrm >= 0 && nrm <= 4.0 * 6.0 + 1e-9);
    for (int64_t z0 = 0; z0 < nz; z0 += 4)
        for (int64_t y0 = 0; y0 < ny; y0 += 8)
            for (int64_t x0 = 0; x0 < nx; x0 += 16) {
                bool any = false;
                for (int64_t z = z0; z < std::min(nz, z0 + 4); ++z)
                    for (int64_t y = y0; y < std::min(ny, y0 + 8); ++y)
                        for (int64_t x = x0; x < std::min(nx, x0 + 16); ++x)
                            any |= mask[(size_t)(x + nx * (y + ny * z))] != 0;
                CHECK(brick_has_inside(g, code, x0, y0, z0, 16, 8, 4) == any);
            }
}

static void check_slab(unsigned seed) {
    std::mt19937_64 rng(seed);
    const size_t cap = (size_t)1 << 30;
    Slab sl;
    sl.init(cap);
    struct A {
        size_t off, n;
    };
    std::vector<A> live;
    size_t used = 0;
    for (int step = 0; step < 20000; ++step) {
        const bool do_alloc = live.empty() || (rng() % 3 != 0 && live.size() < 200);
        if (do_alloc) {
            const size_t n = (size_t)(1 + rng() % 4096) * 256;
            size_t off = 0;
            Fence f;
            if (sl.alloc(n, off, f)) {
                CHECK(off % 256 == 0 && off + n <= cap);
                for (const A &a : live) CHECK(off + n <= a.off || a.off + a.n <= off);
                live.push_back({off, n});
                used += n;
            }
        } else {
            const size_t i = rng() % live.size();
            Fence f;
            f.seq[rng() % kMaxLanes] = step;
            sl.release(live[i].off, live[i].n, f);
            used -= live[i].n;
            live[i] = live.back();
            live.pop_back();
        }
        CHECK(sl.used() == used);
        // free ranges never overlap, never touch (they coalesce) and with the live
        // ranges cover the whole capacity
        size_t prev_end = 0, free_total = 0;
        bool first = true, touching = false;
        sl.each_free([&](size_t off, size_t n) {
            if (!first && off <= prev_end) touching = true;
            first = false;
            prev_end = off + n;
            free_total += n;
        });
        CHECK(!touching);
        CHECK(free_total + used == cap);
    }
    for (const A &a : live) sl.release(a.off, a.n, Fence{});
    int ranges = 0;
    sl.each_free([&](size_t off, size_t n) {
        ++ranges;
        CHECK(off == 0 && n == cap);
    });
    CHECK(ranges == 1 && sl.used() == 0);
}

int main() {
    check_svd(30, 100, 1, 0);
    check_svd(60, 40, 2, 0);
    check_svd(1, 7, 3, 0);
    check_svd(9, 1, 4, 0);
    check_svd(12, 12, 5, 3);
    check_svd(100, 64, 6, 0);
    check_masks(19, 13, 5, 0.6, 7);
    check_masks(40, 1, 1, 0.5, 8);
    check_masks(1, 1, 1, 1.0, 9);
    check_masks(33, 17, 9, 0.0, 10);
    check_masks(16, 8, 4, 1.0, 11);
    check_slab(12);
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
