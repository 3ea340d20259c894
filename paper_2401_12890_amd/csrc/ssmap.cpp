// libssmap host side: the C ABI, validation, parameter rules, device memory
// plan and the launch sequence of the LADMM solve (Algorithm 2, Sec. III-E).
#include "../../include/ssmap.h"
#include "internal.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

using namespace ssmap;

namespace ssmap {

int rank_rule(const std::vector<double> &s, int rank) {
    const int k = (int)s.size();
    if (rank == -1) return k;
    if (rank > 0) return rank;
    // tails from the end: tail[r] = sum_{i >= r} s_i^2
    std::vector<double> tail(k + 1, 0.0);
    for (int i = k - 1; i >= 0; --i) tail[i] = tail[i + 1] + s[i] * s[i];
    const double total = tail[0];
    for (int r = 1; r <= k; ++r)
        if (std::sqrt(tail[r]) < kRankTol * std::sqrt(total)) return r;
    return k;
}

double dtd_norm_closed(const Grid &g) {
    // D^T D = 2 (L_x (+) L_y (+) L_z); a path of n voxels has largest
    // Laplacian eigenvalue 2 + 2 cos(pi / n) (0 when n = 1).
    double lam = 0.0;
    for (int64_t n : {g.nx, g.ny, g.nz})
        if (n > 1) lam += 2.0 + 2.0 * std::cos(M_PI / (double)n);
    return 2.0 * lam;
}

// Solve constants of one (dictionary, precision, rank, beta) in float64 and in
// the state type of the mode: a_i = 1/(beta + s_i^2), b_i = s_i^2/(beta + s_i^2)
// (the 1/beta - s_i and beta s_i of Eq. (DictVecSVD)), V_r zero-padded to
// Qp x RP, U_r, the singular values, and the fused kernel's V operand blocks.
void host_consts(int mode, const std::vector<double> &U, const std::vector<double> &s,
                 const std::vector<double> &V, int kmin, int P, int Q, int Qp, int r, int RP,
                 double beta, bool fused, HostConsts &out) {
    out.Vh.assign((size_t)Qp * RP, 0.0);
    out.Ur.assign((size_t)P * r, 0.0);
    out.sig.assign(RP, 0.0);
    out.a.assign(RP, 0.0);
    std::vector<double> bh(RP, 0.0);
    for (int q = 0; q < Q; ++q)
        for (int i = 0; i < r; ++i) out.Vh[(size_t)q * RP + i] = V[(size_t)q * kmin + i];
    for (int p = 0; p < P; ++p)
        for (int i = 0; i < r; ++i) out.Ur[(size_t)p * r + i] = U[(size_t)p * kmin + i];
    for (int i = 0; i < r; ++i) {
        const double s2 = s[i] * s[i];
        out.sig[i] = s[i];
        out.a[i] = 1.0 / (beta + s2);
        bh[i] = s2 / (beta + s2);
    }
    auto as_bytes = [](const auto &v, std::vector<uint8_t> &dst) {
        dst.resize(v.size() * sizeof(v[0]));
        if (!v.empty()) std::memcpy(dst.data(), v.data(), dst.size());
    };
    out.Vop.clear();
    if (mode == MODE_FP64) {
        as_bytes(out.Vh, out.V);
        as_bytes(bh, out.b);
    } else {
        as_bytes(std::vector<float>(out.Vh.begin(), out.Vh.end()), out.V);
        as_bytes(std::vector<float>(bh.begin(), bh.end()), out.b);
    }
    if (!fused) return;
    if (mode == MODE_BF16X3) {
        std::vector<uint16_t> v16;
        fused_operands_bf16(out.Vh, Qp, RP, v16);
        as_bytes(v16, out.Vop);
    } else {
        std::vector<double> v64;
        fused_operands(out.Vh, Qp, RP, mode == MODE_FP64, fused_tail(mode, RP, r), v64);
        if (mode == MODE_FP64) as_bytes(v64, out.Vop);
        else as_bytes(std::vector<float>(v64.begin(), v64.end()), out.Vop);
    }
}

}  // namespace ssmap

namespace {

struct Fail {
    ssmap_status status;
    std::string msg;
};

[[noreturn]] void fail(ssmap_status st, const std::string &msg) { throw Fail{st, msg}; }

std::string g_create_error;            // last ssmap_create failure (no context yet)

}  // namespace

struct ssmap_ctx {
    int P = 0, Q = 0, kmin = 0, Qp = 0, nchunk = 0;
    Grid g{};
    int device = 0;
    std::vector<double> U, s, V;          // thin SVD: U (P x k), s (k), V (Q x k)
    double dtd_norm = 0.0;
    bool poisoned = false;
    std::string err;
    ssmap_stats stats{};
    // device buffers by name; kept until destroy and grown on demand
    std::map<std::string, std::pair<void *, size_t>> bufs;
    size_t held = 0;
    // aux of the last solve
    bool aux_valid = false;
    int aux_mode = 0;
    int aux_iters = 0;
    int aux_ld = 0;                       // aux_f / aux_d: 0 chunked state; > 0 voxel-major float32 rows
    void *aux_f = nullptr, *aux_d = nullptr;
    // masked voxel set (empty code: the whole box)
    std::vector<uint8_t> code;
    int64_t inside = 0;
    hipEvent_t ev[6] = {};
    double *host_stats = nullptr;         // pinned ST_COUNT doubles
    std::vector<hipEvent_t> gemm_ev;      // GEMM path: 3 timing events per iteration
    // allocation-free solve in progress: every buffer of the solve is carved
    // from the device's static scratch array instead of being allocated
    struct Arena {
        bool on = false;
        char *base = nullptr;
        size_t cap = 0, used = 0;
        std::map<std::string, std::pair<void *, size_t>> bufs;
    } arena;
    void *scratch = nullptr;              // this device's scratch array (NULL: lookup failed)
    bool has_ref = false;                 // a reference map f* for DFCS is on the device ("fstar")
    bool has_init = false;                // an initial iterate for warm starts is set
    bool init_z = false, init_d = false;  // z^0 / d^0 given ("init_z", "init_d"), else zeros
    LibGemm *lg = nullptr;                // exact-rank path: the library products (hipBLASLt)
    bool lg_tried = false;
    hipError_t scratch_err = hipSuccess;
};

namespace {

void hip_check(ssmap_ctx *c, hipError_t e, const char *what) {
    if (e != hipSuccess) {
        if (c) c->poisoned = true;
        fail(SSMAP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
}
#define HIPC(ctx, call) hip_check(ctx, (call), #call)

size_t budget_bytes() {
    const char *env = std::getenv("SSMAP_HBM_BUDGET");
    if (!env || !*env) return (size_t)-1;
    char *end = nullptr;
    const double v = std::strtod(env, &end);
    if (!(v >= 0)) return (size_t)-1;
    return (size_t)v;
}

size_t align256(size_t b) { return (std::max<size_t>(b, 256) + 255) / 256 * 256; }

// An allocation-free solve: the named buffer from the scratch array (the same
// name gives the same range for the rest of the solve).
void *carve(ssmap_ctx *c, const std::string &name, size_t bytes) {
    auto &A = c->arena;
    auto it = A.bufs.find(name);
    if (it != A.bufs.end() && it->second.second >= bytes) return it->second.first;
    const size_t sz = align256(bytes);
    if (A.used + sz > A.cap)
        fail(SSMAP_EINVAL, "allocation-free solve needs more than the " + std::to_string(A.cap) +
                               " bytes of the scratch array (" + name + ")");
    void *p = A.base + A.used;
    A.used += sz;
    A.bufs[name] = {p, bytes};
    return p;
}

// Make sure the named buffer holds at least `bytes`; returns the pointer.
void *ensure(ssmap_ctx *c, const std::string &name, size_t bytes) {
    if (c->arena.on) return carve(c, name, bytes);
    bytes = std::max<size_t>(bytes, 256);
    auto it = c->bufs.find(name);
    if (it != c->bufs.end() && it->second.second >= bytes) return it->second.first;
    size_t extra = bytes - (it != c->bufs.end() ? it->second.second : 0);
    if (c->held + extra > budget_bytes())
        fail(SSMAP_ENOMEM, "device memory budget exceeded (SSMAP_HBM_BUDGET) for " + name);
    if (it != c->bufs.end()) {
        HIPC(c, hipFree(it->second.first));
        c->held -= it->second.second;
        c->bufs.erase(it);
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        fail(SSMAP_ENOMEM, "hipMalloc failed for " + name);
    }
    HIPC(c, e);
    c->bufs[name] = {p, bytes};
    c->held += bytes;
    return p;
}

// The four timing events of GEMM-path iteration k (created on first use): before
// and after each of the two products.
hipEvent_t *gemm_events(ssmap_ctx *c, int k) {
    const size_t need = 4 * (size_t)(k + 1);
    while (c->gemm_ev.size() < need) {
        hipEvent_t e = nullptr;
        HIPC(c, hipEventCreate(&e));
        c->gemm_ev.push_back(e);
    }
    return &c->gemm_ev[4 * (size_t)k];
}

// Device copy of the mask codes (NULL without a mask).
const uint8_t *mask_dev(ssmap_ctx *c) {
    if (c->code.empty()) return nullptr;
    auto it = c->bufs.find("code");
    return it == c->bufs.end() ? nullptr : (const uint8_t *)it->second.first;
}

// Device copy of the reference map f* (NULL when none is set).
const double *ref_dev(ssmap_ctx *c) {
    if (!c->has_ref) return nullptr;
    auto it = c->bufs.find("fstar");
    return it == c->bufs.end() ? nullptr : (const double *)it->second.first;
}

// Plan check before any allocation of a solve: fail early with ENOMEM (or, for an
// allocation-free solve, EINVAL when the scratch array is too small).
void plan_check(ssmap_ctx *c, const std::vector<std::pair<std::string, size_t>> &need) {
    if (c->arena.on) {
        size_t total = c->arena.used;
        for (auto &kv : need)
            if (!c->arena.bufs.count(kv.first)) total += align256(kv.second);
        if (total > c->arena.cap)
            fail(SSMAP_EINVAL, "allocation-free solve needs " + std::to_string(total) +
                                   " device bytes, above the " + std::to_string(c->arena.cap) +
                                   "-byte scratch array");
        return;
    }
    size_t extra = 0;
    for (auto &kv : need) {
        auto it = c->bufs.find(kv.first);
        const size_t have = it == c->bufs.end() ? 0 : it->second.second;
        if (kv.second > have) extra += kv.second - have;
    }
    if (c->held + extra > budget_bytes())
        fail(SSMAP_ENOMEM, "solve needs " + std::to_string(c->held + extra) +
                               " device bytes, above SSMAP_HBM_BUDGET");
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) == hipSuccess && extra > freeb)
        fail(SSMAP_ENOMEM, "solve needs " + std::to_string(extra) + " more device bytes than free");
}

struct Plan {
    int mode, r, RP;
    double xi, tau, beta, lam;
    bool fused;
    bool split;        // small problems: the fused step split over chunks (kernels_split.hip)
    bool gemm;         // exact-rank path: contractions as GEMMs (ranks above 32)
    int Qg, Rg;        // its padded node and rank counts (multiples of 128)
};

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return (double)ms;
}

void validate_steps(ssmap_ctx *c, double lambda, const ssmap_steps *st, int iters) {
    if (!st) fail(SSMAP_EINVAL, "steps is NULL");
    if (!(std::isfinite(lambda) && lambda >= 0)) fail(SSMAP_EINVAL, "lambda must be finite and >= 0");
    if (!(std::isfinite(st->beta) && st->beta > 0)) fail(SSMAP_EINVAL, "beta must be finite and > 0");
    if (!std::isfinite(st->xi_p)) fail(SSMAP_EINVAL, "xi_p must be finite");
    if (iters < 0) fail(SSMAP_EINVAL, "iters must be >= 0");
    if (st->rank < -1 || st->rank > c->kmin) fail(SSMAP_EINVAL, "rank must be in [-1, min(P,Q)]");
    if (st->precision < SSMAP_FP64 || st->precision > SSMAP_BF16X3)
        fail(SSMAP_EINVAL, "unknown precision");
    if (st->check_every < 0) fail(SSMAP_EINVAL, "check_every must be >= 0");
    if (st->kernel < SSMAP_KERNEL_AUTO || st->kernel > SSMAP_KERNEL_SPLIT)
        fail(SSMAP_EINVAL, "unknown kernel");
    if (!(std::isfinite(st->stop_tol) && st->stop_tol >= 0))
        fail(SSMAP_EINVAL, "stop_tol must be finite and >= 0");
    if (st->stop_tol > 0 && (st->check_every == 0 || (st->flags & SSMAP_KEEP_AUX)))
        fail(SSMAP_EINVAL, "stop_tol needs check_every > 0 and no SSMAP_KEEP_AUX");
    if ((st->flags & SSMAP_WARM_START) && !c->has_init)
        fail(SSMAP_EINVAL, "SSMAP_WARM_START without an initial iterate (ssmap_set_initial)");
}

// Bricks of a grid for a brick shape (without a mask).
int64_t brick_count(const Grid &g, FusedShape sh) {
    return ((g.nx + 15) / 16) * ((g.ny + sh.ty - 1) / sh.ty) * ((g.nz + sh.tz - 1) / sh.tz);
}
// AUTO takes the chunk split up to this many bricks and chunks (a 32 x 32 grid with
// Q = 100 is 8 bricks of 16 x 8 and 7 chunks)
constexpr int64_t kSplitMaxBricks = 32;
constexpr int kSplitMaxChunks = 32;

// allow_split: false for batches, whose shared launches run the fused kernel.
Plan make_plan(ssmap_ctx *c, double lambda, const ssmap_steps *st, bool allow_split = true) {
    Plan p{};
    p.mode = st->precision;
    p.r = rank_rule(c->s, st->rank);
    p.beta = st->beta;
    p.lam = lambda;
    p.xi = st->xi_p > 0 ? st->xi_p : kXiFactor * lambda * c->dtd_norm + kEpsXi;
    p.tau = 1.0 / (p.xi + p.beta);
    p.RP = ((p.r + 15) / 16) * 16;
    const bool can_fuse = fused_supported(p.mode, p.RP, c->g.N);
    if (st->kernel == SSMAP_KERNEL_FUSED && !can_fuse)
        fail(SSMAP_EINVAL, "no fused kernel for this precision and rank");
    p.fused = st->kernel == SSMAP_KERNEL_FUSED || (st->kernel == SSMAP_KERNEL_AUTO && can_fuse);
    // GEMM path: float32 / bf16x3 without aux output or primal residual (f is never
    // formed there); AUTO takes it where no fused kernel exists
    const bool gemm_ok = p.mode != MODE_FP64 && !(st->flags & (SSMAP_MONITOR_PRIMAL | SSMAP_WARM_START));
    if (st->kernel == SSMAP_KERNEL_GEMM && !gemm_ok)
        fail(SSMAP_EINVAL, "the GEMM path runs float32 or bf16x3 without primal residual or warm start");
    p.gemm = st->kernel == SSMAP_KERNEL_GEMM || (st->kernel == SSMAP_KERNEL_AUTO && !can_fuse && gemm_ok);
    // Chunk split: float64 / float32 grids with few bricks and short spectra, where
    // one workgroup per brick would leave most CUs idle (no aux output or primal
    // residual: f and d are formed from the fused r-vector state)
    const int64_t esz = p.mode == MODE_FP64 ? 8 : 4;
    const bool split_ok = can_fuse && p.mode != MODE_BF16X3 && c->nchunk >= 2 &&
                          (int64_t)c->nchunk * p.RP * c->g.N * esz < ((int64_t)1 << 31) &&
                          !(st->flags & (SSMAP_KEEP_AUX | SSMAP_MONITOR_PRIMAL | SSMAP_WARM_START));
    if (st->kernel == SSMAP_KERNEL_SPLIT && !split_ok)
        fail(SSMAP_EINVAL, "the split kernel runs float64 or float32 with at least two chunks, "
                           "no aux output, no primal residual and no warm start");
    p.split = st->kernel == SSMAP_KERNEL_SPLIT ||
              (st->kernel == SSMAP_KERNEL_AUTO && allow_split && split_ok && c->nchunk <= kSplitMaxChunks &&
               brick_count(c->g, default_shape(p.mode, c->g)) <= kSplitMaxBricks);
    if (p.split) p.fused = true;
    p.Qg = (c->Q + 127) / 128 * 128;
    p.Rg = (p.r + 127) / 128 * 128;
    return p;
}

// Compute units of the current device (0 when unknown), read once per device.
int current_device_cus() {
    static std::atomic<int> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    int n = cus[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) n = 0;
        cus[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

// The brick shape of a plan's launches: the default shape, except for the chunk
// split on planar grids, which takes the thinnest of 16 x {2, 4, 8} bricks whose
// (brick, chunk) workgroups (one per CU) still fit the device at once, so that an
// iteration's loads are spread over more CUs (a 32 x 32 grid with 7 chunks: 224
// workgroups of 16 x 2 voxels instead of 56 of 16 x 8).
FusedShape plan_shape(const ssmap_ctx *c, const Plan &pl) {
    const FusedShape def = default_shape(pl.mode, c->g);
    if (!pl.split || c->g.nz != 1) return def;
    const int dc = current_device_cus();
    const int64_t cus = dc > 0 ? dc : 256;
    for (int ty : {2, 4, 8})
        if (brick_count(c->g, FusedShape{ty, 1}) * c->nchunk <= cus) return FusedShape{ty, 1};
    return def;
}

// ---------------------------------------------------------------- solve phases
// A solve is prepare (per-solve coefficients, operand images, projection a1,
// state initialisation), the iteration loop (a2..a7) and finish (a8). The
// single-problem entry points run all three; a batch prepares every job,
// runs one loop whose fused launches cover all jobs of a class, and
// finishes every job.
struct Prepared {
    Plan pl;
    IterArgs a{};             // z / znew of iteration 0
    void *z[2] = {nullptr, nullptr};
    bool monitor = false, aux = false, primal = false;
    bool warm = false;            // z^0, d^0 from ssmap_set_initial
    double *V64 = nullptr, *t = nullptr, *mperp2 = nullptr, *partial = nullptr, *stat = nullptr,
           *sig = nullptr;
    const double *fstar = nullptr;
    // f and d around an iteration (aux output, primal residual): d^k is kept in dbuf
    // once known; tbuf takes the other pass's values (see step_job)
    void *auxA = nullptr, *auxB = nullptr;
    mutable void *dbuf = nullptr, *tbuf = nullptr;
    double *monpart = nullptr;    // fused path: per-brick (z^{k+1} - z^k)^2 of a monitored iteration
    int ntiles = 0;
    // chunk split: partials of y (two iterations), s^k = y^{k-1} + w^{k-1} (two)
    void *sp[2] = {nullptr, nullptr}, *ss[2] = {nullptr, nullptr};
    const void *dM = nullptr;
    int iters = 0;
    double stop_tol = 0.0;
    int check_every = 0;
    // checks read after the run (no stopping rule): each check's sums go to their own
    // slot of mhist (ST_COUNT doubles each); mchecks holds the iteration of each slot
    bool defer = false;
    double *mhist = nullptr;
    mutable std::vector<int> mchecks;
    // GEMM path (voxel-major, padded): z ping-pong; s = y + w; w (float32 operand);
    // a.h; bf16 splits; constants
    float *gz[2] = {nullptr, nullptr}, *gs = nullptr, *gw = nullptr, *gah = nullptr, *gb = nullptr;
    uint16_t *gzs = nullptr, *gws = nullptr;
    const void *gAu = nullptr, *gAy = nullptr;
    bool glib = false;            // products by the library (hipBLASLt), epilogues as passes
    float *gU = nullptr, *gY = nullptr;   // their results: u (N x Qg), y (N x Rg)
    int nseg = 2;                 // bf16 split segments per row (3 for the library products)
};

// Monitor checks of a solve: after every check_every-th iteration and the last.
int monitor_checks(const Prepared &P) {
    if (P.check_every <= 0 || P.iters <= 0) return 0;
    return P.iters / P.check_every + (P.iters % P.check_every != 0);
}

IterArgs args_for(const Prepared &P, int k) {
    IterArgs a = P.a;
    a.z = P.z[k & 1];
    a.znew = P.z[(k & 1) ^ 1];
    return a;
}

// Projection and state initialisation only (used again after autotuning).
void init_state(ssmap_ctx *c, Prepared &P, hipStream_t s) {
    const Plan &pl = P.pl;
    const int64_t N = c->g.N;
    const size_t esz = pl.mode == MODE_FP64 ? 8 : 4;
    int *bad = (int *)ensure(c, "bad", 256);
    launch_zero(bad, 1, 4, s);
    launch_project(pl.mode, P.dM, c->P, (const double *)ensure(c, "Ur", (size_t)c->P * pl.r * 8),
                   P.sig, (const double *)ensure(c, "acoef", (size_t)pl.RP * 8), pl.r, pl.RP, N,
                   P.t, P.mperp2, (void *)P.a.ah, P.a.w, P.a.y, bad, mask_dev(c), s);
    launch_zero(P.z[0], (size_t)c->Qp * N, (int)esz, s);
    launch_zero(P.z[1], (size_t)c->Qp * N, (int)esz, s);
    if (P.aux || P.primal) {
        launch_zero(P.auxA, (size_t)c->Qp * N, (int)esz, s);
        launch_zero(P.auxB, (size_t)c->Qp * N, (int)esz, s);
    }
    if (pl.split) {          // y^0 = 0 (its partials), s^0 = y^{-1} + w^{-1} = 0: then w^0 = a.h
        launch_zero(P.sp[0], (size_t)c->nchunk * pl.RP * N, (int)esz, s);
        launch_zero(P.ss[0], (size_t)pl.RP * N, (int)esz, s);
    }
    if (P.warm) {            // z^0, y^0, w^0 (and d^0 for the aux bracket) from the initial iterate
        const size_t nq = (size_t)N * c->Q * 8;
        launch_warm(pl.mode, P.a, c->init_z ? (const double *)ensure(c, "init_z", nq) : nullptr,
                    c->init_d ? (const double *)ensure(c, "init_d", nq) : nullptr, P.V64, P.z[0],
                    (P.aux || P.primal) ? P.dbuf : nullptr, c->Q, s);
    }
    HIPC(c, hipGetLastError());
}

Prepared prepare_gemm(ssmap_ctx *c, Prepared P, hipStream_t s);

Prepared prepare(ssmap_ctx *c, const void *dM, double lambda, const ssmap_steps *st, int iters,
                 hipStream_t s, bool allow_split = true) {
    Prepared P;
    P.pl = make_plan(c, lambda, st, allow_split);
    P.monitor = st->check_every > 0;
    P.check_every = st->check_every;
    P.stop_tol = st->stop_tol;
    P.aux = (st->flags & SSMAP_KEEP_AUX) != 0;
    P.primal = P.monitor && (st->flags & SSMAP_MONITOR_PRIMAL) != 0;
    P.warm = (st->flags & SSMAP_WARM_START) != 0;
    if (P.pl.gemm) {
        P.dM = dM;
        P.iters = iters;
        return prepare_gemm(c, P, s);
    }
    const Plan &pl = P.pl;
    P.dM = dM;
    P.iters = iters;
    const int64_t N = c->g.N;
    const int Pm = c->P, Q = c->Q, Qp = c->Qp, r = pl.r, RP = pl.RP;
    const size_t esz = pl.mode == MODE_FP64 ? 8 : 4;
    const size_t zbytes = (size_t)Qp * N * esz;
    const size_t rbytes = (size_t)RP * N * esz;

    std::vector<std::pair<std::string, size_t>> need = {
        {"z0", zbytes}, {"z1", zbytes}, {"w", rbytes}, {"y", rbytes}, {"ah", rbytes},
        {"V", (size_t)Qp * RP * esz}, {"b", (size_t)RP * esz}, {"Ur", (size_t)Pm * r * 8},
        {"sig", (size_t)RP * 8}, {"acoef", (size_t)RP * 8}, {"bad", 256}};
    if (P.monitor || P.warm) need.push_back({"V64", (size_t)Qp * RP * 8});
    if (P.monitor) {
        need.push_back({"t", (size_t)r * N * 8});
        need.push_back({"mperp2", (size_t)N * 8});
        need.push_back({"partial", (size_t)kMonitorBlocks * ST_COUNT * 8});
        need.push_back({"stat", (size_t)ST_COUNT * 8});
        need.push_back({"mhist", (size_t)SSMAP_MAX_HIST * ST_COUNT * 8});
    }
    if (P.aux || P.primal) {
        need.push_back({"auxA", zbytes});
        need.push_back({"auxB", zbytes});
    }
    if (pl.fused) {
        need.push_back({"Vop", (size_t)c->nchunk * 8 * RP * 64 * 2});
        // launch plan: two descriptors and at most this many bricks
        const FusedShape sh = plan_shape(c, pl);
        const size_t nb = (size_t)((c->g.nx + 15) / 16) * ((c->g.ny + sh.ty - 1) / sh.ty) *
                          ((c->g.nz + sh.tz - 1) / sh.tz);
        need.push_back({"jobs", 2 * sizeof(IterArgs)});
        need.push_back({"tiles", nb * sizeof(TileRef)});
        if (P.monitor) need.push_back({"monpart", nb * 8});
    }
    if (pl.split)
        for (const char *nm : {"sp0", "sp1"}) need.push_back({nm, (size_t)c->nchunk * rbytes});
    if (pl.split)
        for (const char *nm : {"ss0", "ss1"}) need.push_back({nm, rbytes});
    if (pl.mode == MODE_BF16X3) {
        need.push_back({"Vhi", (size_t)Qp * RP * 2});
        need.push_back({"Vlo", (size_t)Qp * RP * 2});
    }
    plan_check(c, need);
    P.z[0] = ensure(c, "z0", zbytes);
    P.z[1] = ensure(c, "z1", zbytes);
    void *w = ensure(c, "w", rbytes), *y = ensure(c, "y", rbytes), *ah = ensure(c, "ah", rbytes);
    void *Vd = ensure(c, "V", (size_t)Qp * RP * esz);
    void *bd = ensure(c, "b", (size_t)RP * esz);
    double *Ur = (double *)ensure(c, "Ur", (size_t)Pm * r * 8);
    P.sig = (double *)ensure(c, "sig", (size_t)RP * 8);
    double *acoef = (double *)ensure(c, "acoef", (size_t)RP * 8);

    // ---- per-solve coefficients (float64 on the host), Sec. III-F rules
    HostConsts hc;
    host_consts(pl.mode, c->U, c->s, c->V, c->kmin, Pm, Q, Qp, r, RP, pl.beta, pl.fused, hc);
    HIPC(c, hipMemcpyAsync(Vd, hc.V.data(), hc.V.size(), hipMemcpyHostToDevice, s));
    HIPC(c, hipMemcpyAsync(bd, hc.b.data(), hc.b.size(), hipMemcpyHostToDevice, s));
    HIPC(c, hipMemcpyAsync(Ur, hc.Ur.data(), hc.Ur.size() * 8, hipMemcpyHostToDevice, s));
    HIPC(c, hipMemcpyAsync(P.sig, hc.sig.data(), RP * 8, hipMemcpyHostToDevice, s));
    HIPC(c, hipMemcpyAsync(acoef, hc.a.data(), RP * 8, hipMemcpyHostToDevice, s));
    void *Vhi = nullptr, *Vlo = nullptr;
    if (pl.mode == MODE_BF16X3) {
        Vhi = ensure(c, "Vhi", (size_t)Qp * RP * 2);
        Vlo = ensure(c, "Vlo", (size_t)Qp * RP * 2);
        launch_split_bf16((const float *)Vd, (uint16_t *)Vhi, (uint16_t *)Vlo, (size_t)Qp * RP, s);
    }
    void *Vop = nullptr;
    if (pl.fused) {
        Vop = ensure(c, "Vop", hc.Vop.size());
        HIPC(c, hipMemcpyAsync(Vop, hc.Vop.data(), hc.Vop.size(), hipMemcpyHostToDevice, s));
    }
    if (P.monitor || P.warm) {
        P.V64 = (double *)ensure(c, "V64", (size_t)Qp * RP * 8);
        HIPC(c, hipMemcpyAsync(P.V64, hc.Vh.data(), hc.Vh.size() * 8, hipMemcpyHostToDevice, s));
    }
    if (P.monitor) {
        P.t = (double *)ensure(c, "t", (size_t)r * N * 8);
        P.mperp2 = (double *)ensure(c, "mperp2", (size_t)N * 8);
        P.partial = (double *)ensure(c, "partial", (size_t)kMonitorBlocks * ST_COUNT * 8);
        P.stat = (double *)ensure(c, "stat", (size_t)ST_COUNT * 8);
        P.defer = P.stop_tol <= 0 && monitor_checks(P) <= SSMAP_MAX_HIST;
        if (P.defer) P.mhist = (double *)ensure(c, "mhist", (size_t)SSMAP_MAX_HIST * ST_COUNT * 8);
        P.fstar = ref_dev(c);
        if (pl.fused) {
            const FusedShape sh = plan_shape(c, pl);
            const size_t nb = (size_t)((c->g.nx + 15) / 16) * ((c->g.ny + sh.ty - 1) / sh.ty) *
                              ((c->g.nz + sh.tz - 1) / sh.tz);
            P.monpart = (double *)ensure(c, "monpart", nb * 8);
        }
    }
    if (P.aux || P.primal) {
        P.auxA = ensure(c, "auxA", zbytes);
        P.auxB = ensure(c, "auxB", zbytes);
    }
    P.dbuf = P.auxA;
    P.tbuf = P.auxB;
    if (pl.split) {
        const char *names[2][2] = {{"sp0", "sp1"}, {"ss0", "ss1"}};
        void **dst[2] = {P.sp, P.ss};
        for (int b = 0; b < 2; ++b)
            for (int k = 0; k < 2; ++k)
                dst[b][k] = ensure(c, names[b][k], b == 0 ? (size_t)c->nchunk * rbytes : rbytes);
    }
    HIPC(c, hipStreamSynchronize(s));         // host staging vectors are locals

    IterArgs &a = P.a;
    a.w = w;
    a.y = y;
    a.ah = ah;
    a.V = Vd;
    a.Vhi = Vhi;
    a.Vlo = Vlo;
    a.bcoef = bd;
    a.Vu = Vop;
    a.r = r;
    a.RP = RP;
    a.nchunk = c->nchunk;
    a.g = c->g;
    a.tau = pl.tau;
    a.lam2 = 2.0 * pl.lam;
    a.beta = pl.beta;
    a.code = mask_dev(c);

    ssmap_stats &S = c->stats;
    const double setup = S.setup_ms;
    std::memset(&S, 0, sizeof(S));
    S.setup_ms = setup;
    S.rank = r;
    S.rank_padded = RP;
    S.precision = pl.mode;
    S.kernel = pl.split ? SSMAP_KERNEL_SPLIT : pl.fused ? SSMAP_KERNEL_FUSED : SSMAP_KERNEL_UNFUSED;
    S.xi_p = pl.xi;
    S.tau = pl.tau;
    S.dtd_norm = c->dtd_norm;
    S.sigma_max = c->s.empty() ? 0.0 : c->s[0];
    c->aux_valid = false;

    // ---- a1: data projection, state initialisation (z^0 = 0, w^0 = a.h, y^0 = 0)
    HIPC(c, hipEventRecord(c->ev[0], s));
    init_state(c, P, s);
    HIPC(c, hipEventRecord(c->ev[1], s));
    int badh = 0;
    HIPC(c, hipMemcpyAsync(&badh, ensure(c, "bad", 256), 4, hipMemcpyDeviceToHost, s));
    HIPC(c, hipStreamSynchronize(s));
    if (badh) fail(SSMAP_ENONFINITE, "M holds a NaN or Inf");
    return P;
}

// ---- exact-rank GEMM path: constants, projection and state in its layouts
Prepared prepare_gemm(ssmap_ctx *c, Prepared P, hipStream_t s) {
    const Plan &pl = P.pl;
    const int64_t N = c->g.N;
    const int Pm = c->P, Q = c->Q, Qp = c->Qp, r = pl.r, RP = pl.RP, Qg = pl.Qg, Rg = pl.Rg;
    const bool bf = pl.mode == MODE_BF16X3;
    const int Ku = bf ? 3 * Rg : Rg, Ky = bf ? 3 * Qg : Qg;
    const size_t esA = bf ? 2 : 4;
    const size_t zb = (size_t)N * Qg * 4, rb = (size_t)N * Rg * 4, tb = (size_t)N * RP * 4;
    // the library products when hipBLASLt has an algorithm for both shapes
    if (!c->lg_tried) {
        c->lg = libgemm_create();
        c->lg_tried = true;
        (void)hipGetLastError();
    }
    P.glib = c->lg && libgemm_tn(c->lg, bf, nullptr, nullptr, nullptr, Qg, N, Ku, s) &&
             libgemm_tn(c->lg, bf, nullptr, nullptr, nullptr, Rg, N, Ky, s);
    P.nseg = P.glib ? 3 : 2;
    // f and d need u^k, which only the library products leave in memory
    if (P.aux && !P.glib)
        fail(SSMAP_EINVAL, "aux output on the GEMM path needs the hipBLASLt products "
                           "(none for this shape): use SSMAP_KERNEL_UNFUSED");
    std::vector<std::pair<std::string, size_t>> need = {
        {"gz0", zb}, {"gz1", zb}, {"gs", rb}, {"gah", rb}, {"gt0", tb}, {"gt1", tb},
        {"gb", (size_t)Rg * 4}, {"gAu", (size_t)Qg * Ku * esA}, {"gAy", (size_t)Rg * Ky * esA},
        {"Ur", (size_t)Pm * r * 8}, {"sig", (size_t)RP * 8}, {"acoef", (size_t)RP * 8}, {"bad", 256}};
    if (bf) {
        need.push_back({"gzs", (size_t)N * P.nseg * Qg * 2});
        need.push_back({"gws", (size_t)N * P.nseg * Rg * 2});
    } else {
        need.push_back({"gw", rb});
    }
    if (P.glib) {
        need.push_back({"gU", zb});
        need.push_back({"gY", rb});
    }
    if (P.aux) {
        need.push_back({"gaux0", zb});
        need.push_back({"gaux1", zb});
    }
    if (P.monitor) {
        need.push_back({"t", (size_t)r * N * 8});
        need.push_back({"mperp2", (size_t)N * 8});
        need.push_back({"V64", (size_t)Qg * RP * 8});
        need.push_back({"partial", (size_t)kMonitorBlocks * ST_COUNT * 8});
        need.push_back({"stat", (size_t)ST_COUNT * 8});
        need.push_back({"mhist", (size_t)SSMAP_MAX_HIST * ST_COUNT * 8});
    }
    plan_check(c, need);
    for (int k = 0; k < 2; ++k) P.gz[k] = (float *)ensure(c, k ? "gz1" : "gz0", zb);
    if (P.aux) {                  // f and d around the last two iterations (voxel-major)
        P.dbuf = ensure(c, "gaux0", zb);
        P.tbuf = ensure(c, "gaux1", zb);
        launch_zero(P.dbuf, (size_t)N * Qg, 4, s);
        launch_zero(P.tbuf, (size_t)N * Qg, 4, s);
    }
    P.gs = (float *)ensure(c, "gs", rb);
    P.gah = (float *)ensure(c, "gah", rb);
    // rank-major projection temporaries: a.h (= w^0) and y^0
    float *gt0 = (float *)ensure(c, "gt0", tb), *gt1 = (float *)ensure(c, "gt1", tb);
    P.gb = (float *)ensure(c, "gb", (size_t)Rg * 4);
    if (bf) {
        P.gzs = (uint16_t *)ensure(c, "gzs", (size_t)N * P.nseg * Qg * 2);
        P.gws = (uint16_t *)ensure(c, "gws", (size_t)N * P.nseg * Rg * 2);
    } else {
        P.gw = (float *)ensure(c, "gw", rb);
    }
    void *Au = ensure(c, "gAu", (size_t)Qg * Ku * esA), *Ay = ensure(c, "gAy", (size_t)Rg * Ky * esA);
    double *Ur = (double *)ensure(c, "Ur", (size_t)Pm * r * 8);
    P.sig = (double *)ensure(c, "sig", (size_t)RP * 8);
    double *acoef = (double *)ensure(c, "acoef", (size_t)RP * 8);

    // constants: A of u (Qg x Ku, row-major) and A of y (Rg x Ky); bf16x3 concatenates
    // hi | hi | lo along K against the operands' hi | lo | hi
    HostConsts hc;
    host_consts(pl.mode, c->U, c->s, c->V, c->kmin, Pm, Q, Qp, r, RP, pl.beta, false, hc);
    if (P.monitor) {
        // float64 V_r for the monitor's contraction, Qg x RP (rows beyond Qp are zero)
        P.V64 = (double *)ensure(c, "V64", (size_t)Qg * RP * 8);
        std::vector<double> v64((size_t)Qg * RP, 0.0);
        std::copy(hc.Vh.begin(), hc.Vh.end(), v64.begin());
        HIPC(c, hipMemcpyAsync(P.V64, v64.data(), v64.size() * 8, hipMemcpyHostToDevice, s));
        P.t = (double *)ensure(c, "t", (size_t)r * N * 8);
        P.mperp2 = (double *)ensure(c, "mperp2", (size_t)N * 8);
        P.partial = (double *)ensure(c, "partial", (size_t)kMonitorBlocks * ST_COUNT * 8);
        P.stat = (double *)ensure(c, "stat", (size_t)ST_COUNT * 8);
        P.defer = P.stop_tol <= 0 && monitor_checks(P) <= SSMAP_MAX_HIST;
        if (P.defer) P.mhist = (double *)ensure(c, "mhist", (size_t)SSMAP_MAX_HIST * ST_COUNT * 8);
        P.fstar = ref_dev(c);
        HIPC(c, hipStreamSynchronize(s));      // v64 is a local
    }
    auto Vf = [&](int q, int i) -> float {
        return (q < Q && i < r) ? (float)hc.Vh[(size_t)q * RP + i] : 0.0f;
    };
    std::vector<float> bg(Rg, 0.0f);
    for (int i = 0; i < r; ++i) bg[i] = (float)(c->s[i] * c->s[i] / (pl.beta + c->s[i] * c->s[i]));
    if (bf) {
        auto bits = [](float x) {
            uint32_t u;
            std::memcpy(&u, &x, 4);
            u += 0x7FFFu + ((u >> 16) & 1u);
            return (uint16_t)(u >> 16);
        };
        auto val = [](uint16_t b) {
            const uint32_t u = (uint32_t)b << 16;
            float x;
            std::memcpy(&x, &u, 4);
            return x;
        };
        std::vector<uint16_t> au((size_t)Qg * Ku), ay((size_t)Rg * Ky);
        for (int q = 0; q < Qg; ++q)
            for (int i = 0; i < Rg; ++i) {
                const float f = Vf(q, i);
                const uint16_t h = bits(f), l = bits(f - val(h));
                au[(size_t)q * Ku + i] = h;
                au[(size_t)q * Ku + Rg + i] = h;
                au[(size_t)q * Ku + 2 * Rg + i] = l;
                ay[(size_t)i * Ky + q] = h;
                ay[(size_t)i * Ky + Qg + q] = h;
                ay[(size_t)i * Ky + 2 * Qg + q] = l;
            }
        HIPC(c, hipMemcpyAsync(Au, au.data(), au.size() * 2, hipMemcpyHostToDevice, s));
        HIPC(c, hipMemcpyAsync(Ay, ay.data(), ay.size() * 2, hipMemcpyHostToDevice, s));
        HIPC(c, hipStreamSynchronize(s));
    } else {
        std::vector<float> au((size_t)Qg * Ku), ay((size_t)Rg * Ky);
        for (int q = 0; q < Qg; ++q)
            for (int i = 0; i < Rg; ++i) {
                au[(size_t)q * Ku + i] = Vf(q, i);
                ay[(size_t)i * Ky + q] = Vf(q, i);
            }
        HIPC(c, hipMemcpyAsync(Au, au.data(), au.size() * 4, hipMemcpyHostToDevice, s));
        HIPC(c, hipMemcpyAsync(Ay, ay.data(), ay.size() * 4, hipMemcpyHostToDevice, s));
        HIPC(c, hipStreamSynchronize(s));
    }
    P.gAu = Au;
    P.gAy = Ay;
    HIPC(c, hipMemcpyAsync(P.gb, bg.data(), Rg * 4, hipMemcpyHostToDevice, s));
    HIPC(c, hipMemcpyAsync(Ur, hc.Ur.data(), hc.Ur.size() * 8, hipMemcpyHostToDevice, s));
    HIPC(c, hipMemcpyAsync(P.sig, hc.sig.data(), RP * 8, hipMemcpyHostToDevice, s));
    HIPC(c, hipMemcpyAsync(acoef, hc.a.data(), RP * 8, hipMemcpyHostToDevice, s));
    HIPC(c, hipStreamSynchronize(s));     // host staging vectors are locals

    ssmap_stats &S = c->stats;
    const double setup = S.setup_ms;
    std::memset(&S, 0, sizeof(S));
    S.setup_ms = setup;
    S.rank = r;
    S.rank_padded = Rg;
    S.precision = pl.mode;
    S.kernel = SSMAP_KERNEL_GEMM;
    S.xi_p = pl.xi;
    S.tau = pl.tau;
    S.dtd_norm = c->dtd_norm;
    S.sigma_max = c->s.empty() ? 0.0 : c->s[0];
    c->aux_valid = false;

    // a1: projection into rank-major temporaries (a.h = w^0, y^0 = 0), then the
    // voxel-major a.h, s^0 = y^0 + w^0 = w^0 and w^0 (float32 or its split); z^0 = 0
    HIPC(c, hipEventRecord(c->ev[0], s));
    int *bad = (int *)ensure(c, "bad", 256);
    launch_zero(bad, 1, 4, s);
    launch_project(pl.mode, P.dM, Pm, Ur, P.sig, acoef, r, RP, N, P.t, P.mperp2, gt0, gt0, gt1,
                   bad, mask_dev(c), s);
    launch_gemm_from_ranks(gt0, RP, P.gah, nullptr, N, Rg, s);
    if (P.glib) {
        P.gU = (float *)ensure(c, "gU", zb);
        P.gY = (float *)ensure(c, "gY", rb);
    }
    launch_gemm_from_ranks(gt0, RP, P.gs, P.gws, N, Rg, s, P.nseg);
    if (!bf) launch_gemm_from_ranks(gt0, RP, P.gw, nullptr, N, Rg, s);
    for (int k = 0; k < 2; ++k) launch_zero(P.gz[k], (size_t)N * Qg, 4, s);
    HIPC(c, hipGetLastError());
    HIPC(c, hipEventRecord(c->ev[1], s));
    int badh = 0;
    HIPC(c, hipMemcpyAsync(&badh, bad, 4, hipMemcpyDeviceToHost, s));
    HIPC(c, hipStreamSynchronize(s));
    if (badh) fail(SSMAP_ENONFINITE, "M holds a NaN or Inf");
    return P;
}

// One GEMM-path iteration k: u = V_r w^k with the z-update as its epilogue, then
// y^{k+1} = V_r^T z^{k+1} with the r-vector recursion as its epilogue. Both
// launches are bracketed by timing events (stats.gemm_ms).
bool wants_f(const Prepared &P, int k);

void step_gemm(ssmap_ctx *c, const Prepared &P, int k, hipStream_t s) {
    const Plan &pl = P.pl;
    const bool bf = pl.mode == MODE_BF16X3;
    const int64_t N = c->g.N;
    const int Qg = pl.Qg, Rg = pl.Rg;
    const float *z = P.gz[k & 1];
    float *zn = P.gz[(k + 1) & 1];
    hipEvent_t *ev = gemm_events(c, k);
    const void *Bu = bf ? (const void *)P.gws : (const void *)P.gw;
    const void *By = bf ? (const void *)P.gzs : (const void *)zn;
    const int Ku = bf ? 3 * Rg : Rg, Ky = bf ? 3 * Qg : Qg;
    if (P.glib) {
        // library products, then the epilogues as passes over u and y
        HIPC(c, hipEventRecord(ev[0], s));
        if (!libgemm_tn(c->lg, bf, P.gAu, Bu, P.gU, Qg, N, Ku, s)) fail(SSMAP_EDEVICE, "hipBLASLt product failed");
        HIPC(c, hipEventRecord(ev[1], s));
        launch_epi_z(P.gU, z, zn, bf ? P.gzs : nullptr, c->g, Qg, pl.tau, 2.0 * pl.lam, pl.beta, mask_dev(c), s);
        // f^{k+1} and d^{k+1} around the last two iterations (as the fused path's
        // bracket; afterwards dbuf holds d^{k+1}, tbuf f^{k+1})
        const bool need_f = wants_f(P, k);
        if (need_f || wants_f(P, k + 1)) {
            launch_gemm_aux(z, P.gU, zn, need_f && k > 0 ? (const float *)P.dbuf : nullptr,
                            need_f ? (float *)P.dbuf : nullptr, (float *)P.tbuf, (size_t)N * Qg, pl.beta, s);
            std::swap(P.dbuf, P.tbuf);
        }
        HIPC(c, hipEventRecord(ev[2], s));
        if (!libgemm_tn(c->lg, bf, P.gAy, By, P.gY, Rg, N, Ky, s)) fail(SSMAP_EDEVICE, "hipBLASLt product failed");
        HIPC(c, hipEventRecord(ev[3], s));
        launch_epi_w(P.gY, N, Rg, P.gah, P.gs, bf ? nullptr : P.gw, bf ? P.gws : nullptr, P.gb, s);
        HIPC(c, hipGetLastError());
        return;
    }
    HIPC(c, hipEventRecord(ev[0], s));
    if (!launch_gemm_u(bf, P.gAu, Bu, Ku, z, zn, P.gzs, c->g, Qg, pl.tau, 2.0 * pl.lam, pl.beta,
                       mask_dev(c), s))
        fail(SSMAP_EINVAL, "GEMM shape not supported");
    HIPC(c, hipEventRecord(ev[1], s));
    HIPC(c, hipEventRecord(ev[2], s));
    if (!launch_gemm_y(bf, P.gAy, By, Ky, N, Rg, P.gah, P.gs, P.gw, P.gws, P.gb, s))
        fail(SSMAP_EINVAL, "GEMM shape not supported");
    HIPC(c, hipEventRecord(ev[3], s));
}

void finish_gemm(ssmap_ctx *c, const Prepared &P, void *dF, hipStream_t s) {
    const int iters = P.iters;
    launch_gemm_output(P.gz[iters & 1], dF, false, c->g.N, c->Q, P.pl.Qg, s);
    HIPC(c, hipGetLastError());
    HIPC(c, hipEventRecord(c->ev[4], s));
    HIPC(c, hipStreamSynchronize(s));
    ssmap_stats &S = c->stats;
    S.iters = iters;
    S.device_bytes = (double)c->held;
    double ms = 0.0;
    for (int k = 0; k < iters; ++k) {
        hipEvent_t *ev = gemm_events(c, k);
        ms += elapsed_ms(ev[0], ev[1]) + elapsed_ms(ev[2], ev[3]);
    }
    S.gemm_ms = ms;
    S.gemm_library = P.glib ? 1 : 0;
    if (P.aux) {
        c->aux_valid = true;
        c->aux_mode = MODE_FP32;
        c->aux_iters = iters;
        c->aux_f = P.tbuf;
        c->aux_d = P.dbuf;
        c->aux_ld = P.pl.Qg;
    }
    const bool bf = P.pl.mode == MODE_BF16X3;
    S.gemm_flops = 2.0 * 2.0 * (double)P.pl.Qg * P.pl.Rg * (bf ? 3.0 : 1.0) * (double)c->g.N * iters;
}

// Device copies of a one-job launch plan: two IterArgs (even / odd
// iterations) and the brick table for the default shape.
FusedLaunch single_launch(ssmap_ctx *c, const Prepared &P, hipStream_t s) {
    FusedLaunch L{};
    L.mode = P.pl.mode;
    L.r = P.pl.r;
    L.RP = P.pl.RP;
    L.shape = plan_shape(c, P.pl);
    std::vector<TileRef> tiles;
    append_tiles(c->g, 0, L.mode, L.shape, tiles, c->code.empty() ? nullptr : &c->code);
    IterArgs two[2] = {args_for(P, 0), args_for(P, 1)};
    IterArgs *dj = (IterArgs *)ensure(c, "jobs", sizeof(two));
    TileRef *dt = (TileRef *)ensure(c, "tiles", tiles.size() * sizeof(TileRef));
    HIPC(c, hipMemcpyAsync(dj, two, sizeof(two), hipMemcpyHostToDevice, s));
    HIPC(c, hipMemcpyAsync(dt, tiles.data(), tiles.size() * sizeof(TileRef), hipMemcpyHostToDevice, s));
    HIPC(c, hipStreamSynchronize(s));
    L.jobs = dj;
    L.tiles = dt;
    L.ntiles = (int)tiles.size();
    L.maxchunk = c->nchunk;
    return L;
}

// Monitoring after iteration k (z^{k+1} against z^k; f^{k+1} when the primal
// residual is asked for, left in tbuf by the bracket of iteration k): the
// reductions, in stream order, into `out` (ST_COUNT doubles on the device).
void monitor_launch(ssmap_ctx *c, const Prepared &P, int k, double *out, hipStream_t s) {
    const Plan &pl = P.pl;
    MonArgs m{};
    if (pl.gemm) {
        m.z = P.gz[(k + 1) & 1];
        m.zprev = P.gz[k & 1];
        m.ld = pl.Qg;
        m.nchunk = pl.Qg / QC;
        if (P.glib) {                // the library product left y^{k+1} = V_r^T z^{k+1} (N x Rg)
            m.y = P.gY;
            m.yld = pl.Rg;
        }
    } else {
        // the iteration left y^{k+1} = V_r^T z^{k+1} in its r-vector state; the fused
        // kernel also summed (z^{k+1} - z^k)^2 per brick
        m.z = P.z[(k + 1) & 1];
        if (pl.split) {              // y^{k+1} exists only as per-chunk partials
            m.zprev = P.z[k & 1];
            m.ypart = P.sp[(k + 1) & 1];
            m.npart = c->nchunk;
        } else if (pl.fused) {
            m.y = P.a.y;
            m.dzpart = P.monpart;
            m.ndz = P.ntiles;
        } else {
            m.y = P.a.y;
            m.zprev = P.z[k & 1];
        }
        m.f = P.primal ? P.tbuf : nullptr;
        m.nchunk = c->nchunk;
    }
    m.fstar = P.fstar;
    m.V64 = P.V64;
    m.sig = P.sig;
    m.t = P.t;
    m.mperp2 = P.mperp2;
    m.r = pl.r;
    m.RP = pl.RP;
    m.Q = c->Q;
    m.g = c->g;
    m.code = mask_dev(c);
    launch_monitor(pl.mode, m, P.partial, out, s);
    HIPC(c, hipGetLastError());
}

// One check's sums `h` (host) after iteration k into the history; ENONFINITE for a
// non-finite iterate. Returns true when the residual stopping rule fires: k + 1 is
// a multiple of check_every and ||z^{k+1} - z^k|| <= stop_tol ||z^{k+1}||.
bool monitor_record(ssmap_ctx *c, const Prepared &P, int k, const double *h) {
    const Plan &pl = P.pl;
    ssmap_stats &S = c->stats;
    if (S.n_hist < SSMAP_MAX_HIST) {
        const int i = S.n_hist++;
        S.hist_iter[i] = k + 1;
        S.hist_objective[i] = 0.5 * h[ST_DATA] + pl.lam * h[ST_REG];
        S.hist_dual[i] = pl.beta * std::sqrt(h[ST_DZ]);
        S.hist_znorm[i] = std::sqrt(h[ST_ZNORM]);
        S.hist_primal[i] = P.primal ? std::sqrt(h[ST_PRIMAL]) : -1.0;
        const double fs = std::sqrt(h[ST_FSTAR]);
        S.hist_dfcs[i] = P.fstar && fs > 0 ? std::sqrt(h[ST_DFCS]) / fs : -1.0;
        S.hist_dfcs_f[i] = P.fstar && P.primal && fs > 0 ? std::sqrt(h[ST_DFCS_F]) / fs : -1.0;
    }
    if (h[ST_NONFINITE] != 0.0 || !std::isfinite(h[ST_DATA]))
        fail(SSMAP_ENONFINITE, "non-finite iterate at iteration " + std::to_string(k + 1));
    return P.stop_tol > 0 && (k + 1) % P.check_every == 0 &&
           std::sqrt(h[ST_DZ]) <= P.stop_tol * std::sqrt(h[ST_ZNORM]);
}

// The check after iteration k. Without a stopping rule it is only enqueued (its
// sums to the next slot of mhist, read by monitor_flush after the run); else the
// host waits for it. Returns true when the stopping rule fires.
bool monitor_step(ssmap_ctx *c, const Prepared &P, int k, hipStream_t s) {
    if (P.defer && P.mchecks.size() < (size_t)SSMAP_MAX_HIST) {
        monitor_launch(c, P, k, P.mhist + P.mchecks.size() * ST_COUNT, s);
        P.mchecks.push_back(k);
        return false;
    }
    monitor_launch(c, P, k, P.stat, s);
    HIPC(c, hipMemcpyAsync(c->host_stats, P.stat, ST_COUNT * 8, hipMemcpyDeviceToHost, s));
    HIPC(c, hipStreamSynchronize(s));
    return monitor_record(c, P, k, c->host_stats);
}

// The deferred checks of a solve, in order, into the history (ENONFINITE names the
// first check that saw a non-finite iterate).
void monitor_flush(ssmap_ctx *c, const Prepared &P, hipStream_t s) {
    if (P.mchecks.empty()) return;
    std::vector<double> h(P.mchecks.size() * ST_COUNT);
    HIPC(c, hipMemcpyAsync(h.data(), P.mhist, h.size() * 8, hipMemcpyDeviceToHost, s));
    HIPC(c, hipStreamSynchronize(s));
    const std::vector<int> ks = std::move(P.mchecks);
    P.mchecks.clear();
    for (size_t i = 0; i < ks.size(); ++i) (void)monitor_record(c, P, ks[i], h.data() + i * ST_COUNT);
}

// One iteration of one job outside a shared launch (unfused kernels, or the
// fused single-job launch with the aux passes around it).
void step_gemm(ssmap_ctx *c, const Prepared &P, int k, hipStream_t s);

// Whether the monitor runs after iteration k (k + 1 iterations done).
bool checked_after(const Prepared &P, int k) {
    return P.monitor && ((k + 1) % P.check_every == 0 || k + 1 == P.iters);
}

// f^{k+1} is formed in iteration k when the monitor after it reports the primal
// residual, or for the aux output after the last iteration.
bool wants_f(const Prepared &P, int k) {
    if (k >= P.iters) return false;
    return (P.primal && checked_after(P, k)) || (P.aux && k == P.iters - 1);
}

void step_job(ssmap_ctx *c, const Prepared &P, const FusedLaunch *L, int k, hipStream_t s) {
    const Plan &pl = P.pl;
    if (pl.gemm) {
        step_gemm(c, P, k, s);
        return;
    }
    if (pl.split) {
        SplitArgs sa{};
        sa.a = args_for(P, k);
        sa.pin = P.sp[k & 1];
        sa.pout = P.sp[(k + 1) & 1];
        sa.sin = P.ss[k & 1];
        sa.sout = P.ss[(k + 1) & 1];
        if (!launch_split(pl.mode, sa, L->shape, L->tiles, L->ntiles, s))
            fail(SSMAP_EINVAL, "no split kernel for this precision and brick shape");
        return;
    }
    IterArgs a = args_for(P, k);
    // f and d around iteration k. The iteration never forms them; when f^{k+1}
    // is wanted (it needs d^k, itself formed around iteration k - 1; d^0 = 0, or
    // the warm start's, which init_state left in dbuf),
    // iteration k is bracketed: t = z^k + V_r w^k and f^{k+1} = t - d^k / beta
    // (over d^k, in place) before it, d^{k+1} = beta (t - z^{k+1}) after it.
    // Afterwards dbuf holds d^{k+1} and tbuf f^{k+1}.
    const bool need_f = wants_f(P, k);
    const bool bracket = need_f || wants_f(P, k + 1);
    void *fbuf = need_f ? P.dbuf : nullptr;
    const void *dprev = need_f && (k > 0 || P.warm) ? P.dbuf : nullptr;   // d^0 = 0 unless warm
    if (bracket) {
        a.dprev = dprev;
        a.fout = fbuf;
        a.dout = P.tbuf;
    }
    if (pl.fused) {
        const size_t cnt = (size_t)c->Qp * c->g.N;
        if (bracket) launch_aux_pre(pl.mode, a, P.tbuf, fbuf, dprev, s);
        FusedLaunch Lk = *L;
        Lk.round = k;
        if (checked_after(P, k)) Lk.mon = P.monpart;
        if (!launch_fused(Lk, s)) fail(SSMAP_EINVAL, "no fused kernel for this brick shape");
        if (bracket) launch_aux_post(pl.mode, P.tbuf, a.znew, pl.beta, cnt, s);
    } else {
        launch_update_unfused(pl.mode, a, s);     // writes f^{k+1} and d^{k+1} itself
        launch_projw_unfused(pl.mode, a, s);
    }
    if (bracket) std::swap(P.dbuf, P.tbuf);
}

void finish_gemm(ssmap_ctx *c, const Prepared &P, void *dF, hipStream_t s);

void finish(ssmap_ctx *c, const Prepared &P, void *dF, hipStream_t s) {
    if (P.pl.gemm) {
        finish_gemm(c, P, dF, s);
        return;
    }
    const int iters = P.iters;
    launch_output(P.pl.mode, P.z[iters & 1], dF, c->Q, c->g.N, false, s);
    HIPC(c, hipGetLastError());
    HIPC(c, hipEventRecord(c->ev[4], s));
    HIPC(c, hipStreamSynchronize(s));
    ssmap_stats &S = c->stats;
    S.iters = iters;
    S.device_bytes = (double)(c->arena.on ? c->arena.used : c->held);
    if (P.aux) {
        c->aux_valid = true;
        c->aux_mode = P.pl.mode;
        c->aux_iters = iters;
        c->aux_f = P.tbuf;
        c->aux_d = P.dbuf;
        c->aux_ld = 0;
    }
}

// The solve of one problem on device buffers (dM, dF in the mode's I/O type).
void solve_impl(ssmap_ctx *c, const void *dM, double lambda, const ssmap_steps *st, int iters,
                void *dF, hipStream_t s) {
    Prepared P = prepare(c, dM, lambda, st, iters, s);
    FusedLaunch L{};
    if (P.pl.fused) L = single_launch(c, P, s);
    P.ntiles = L.ntiles;
    HIPC(c, hipEventRecord(c->ev[2], s));
    for (int k = 0; k < iters; ++k) {
        step_job(c, P, &L, k, s);
        if (checked_after(P, k) && monitor_step(c, P, k, s) && k + 1 < iters) {
            P.iters = k + 1;             // residual stopping rule
            break;
        }
    }
    HIPC(c, hipGetLastError());
    HIPC(c, hipEventRecord(c->ev[3], s));
    monitor_flush(c, P, s);
    finish(c, P, dF, s);
    ssmap_stats &S = c->stats;
    S.project_ms = elapsed_ms(c->ev[0], c->ev[1]);
    S.iterate_ms = elapsed_ms(c->ev[2], c->ev[3]);
    S.output_ms = elapsed_ms(c->ev[3], c->ev[4]);
}

template <typename Fn>
ssmap_status guarded(ssmap_ctx *c, Fn &&fn) {
    try {
        if (c && c->poisoned) fail(SSMAP_EDEVICE, "context poisoned by an earlier device error");
        fn();
        return SSMAP_OK;
    } catch (const Fail &f) {
        if (c) c->err = f.msg;
        else g_create_error = f.msg;
        return f.status;
    } catch (const std::bad_alloc &) {
        if (c) c->err = "host allocation failed";
        else g_create_error = "host allocation failed";
        return SSMAP_ENOMEM;
    } catch (...) {
        if (c) {
            c->err = "unexpected internal error";
            c->poisoned = true;
        } else {
            g_create_error = "unexpected internal error";
        }
        return SSMAP_EDEVICE;
    }
}

void free_ctx(ssmap_ctx *c) {
    if (!c) return;
    for (auto &kv : c->bufs) (void)hipFree(kv.second.first);
    c->bufs.clear();
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->gemm_ev) (void)hipEventDestroy(e);
    libgemm_destroy(c->lg);
    if (c->host_stats) (void)hipHostFree(c->host_stats);
    delete c;
}

// ---------------------------------------------------------------- batches
struct BatchClass {
    int mode = 0, r = 0, RP = 0;
    bool planar = false;
    std::vector<int> jobs;
    FusedShape shape{16, 1};
    int ntiles = 0;
    // monitored members: each member's bricks are one contiguous run of the brick
    // table (tile_off, tile_cnt per member), so the monitored build's per-brick
    // sums of (z^{k+1} - z^k)^2 in `mon` split by job
    std::vector<int> tile_off, tile_cnt;
    double *mon = nullptr;
};

}  // namespace

struct ssmap_batch {
    ssmap_ctx arena;                      // device buffers of the shared launch plans
    std::vector<ssmap_ctx *> jobs;
    std::string err;
    bool poisoned = false;
    ssmap_batch_stats stats{};
    hipEvent_t ev[6] = {};
    // brick shapes chosen by a tuned solve, by class (precision, padded rank,
    // planar, member jobs): later solves of the same classes reuse them
    std::map<std::string, FusedShape> tuned;
};

namespace {

std::string g_batch_create_error;

// Key of a shared-launch class: the fused kernel template (precision and the
// u K-step bucket of the rank) and whether the grids are planar.
int rank_bucket(int r) { return r <= 16 ? 0 : r <= 20 ? 1 : r <= 24 ? 2 : 3; }

void upload_class(ssmap_batch *b, int ci, BatchClass &C, const std::vector<Prepared> &Ps,
                  FusedShape shape, FusedLaunch &L, hipStream_t s) {
    std::vector<IterArgs> args(2 * C.jobs.size());
    std::vector<TileRef> tiles;
    C.tile_off.assign(C.jobs.size(), 0);
    C.tile_cnt.assign(C.jobs.size(), 0);
    bool monitored = false;
    std::vector<std::vector<TileRef>> per(C.jobs.size());
    size_t ntiles = 0;
    for (size_t k = 0; k < C.jobs.size(); ++k) {
        const int j = C.jobs[k];
        args[2 * k] = args_for(Ps[j], 0);                    // even iterations
        args[2 * k + 1] = args_for(Ps[j], 1);                // odd iterations
        append_tiles(b->jobs[j]->g, (int)k, C.mode, shape, per[k],
                     b->jobs[j]->code.empty() ? nullptr : &b->jobs[j]->code);
        ntiles += per[k].size();
        monitored |= Ps[j].monitor;
    }
    // A brick walks all of its job's chunks, so bricks of long spectra take longest.
    // Workgroup b takes brick b when the brick count is not a multiple of 8 (else
    // each XCD takes a contiguous eighth of the table): then the jobs with the most
    // chunks go first, so that the short bricks fill in behind the long ones
    // instead of the long ones running last. A job's bricks stay contiguous.
    std::vector<size_t> order(C.jobs.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    if (ntiles % 8 != 0)
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
            return args[2 * x].nchunk > args[2 * y].nchunk;
        });
    for (size_t k : order) {
        C.tile_off[k] = (int)tiles.size();
        tiles.insert(tiles.end(), per[k].begin(), per[k].end());
        C.tile_cnt[k] = (int)per[k].size();
    }
    ssmap_ctx *A = &b->arena;
    const std::string tag = std::to_string(ci);
    C.mon = monitored ? (double *)ensure(A, "cls_mon" + tag, std::max<size_t>(1, tiles.size()) * 8) : nullptr;
    IterArgs *dj = (IterArgs *)ensure(A, "cls_jobs" + tag, args.size() * sizeof(IterArgs));
    TileRef *dt = (TileRef *)ensure(A, "cls_tiles" + tag, tiles.size() * sizeof(TileRef));
    HIPC(A, hipMemcpyAsync(dj, args.data(), args.size() * sizeof(IterArgs), hipMemcpyHostToDevice, s));
    HIPC(A, hipMemcpyAsync(dt, tiles.data(), tiles.size() * sizeof(TileRef), hipMemcpyHostToDevice, s));
    HIPC(A, hipStreamSynchronize(s));
    L = FusedLaunch{};
    L.mode = C.mode;
    L.r = C.r;
    L.RP = C.RP;
    L.shape = shape;
    L.jobs = dj;
    L.tiles = dt;
    L.ntiles = (int)tiles.size();
    for (const IterArgs &a : args) L.maxchunk = std::max(L.maxchunk, a.nchunk);
}

// One shared launch of iteration k (jobs[2j], jobs[2j+1]: job j's even and
// odd descriptors; a brick names its job by index).
void launch_class(ssmap_batch *b, const FusedLaunch &L, size_t njobs, int k, hipStream_t s,
                  double *mon = nullptr) {
    FusedLaunch Lk = L;
    Lk.round = k;
    Lk.mon = mon;
    if (!launch_fused(Lk, s)) fail(SSMAP_EINVAL, "no fused kernel for this brick shape");
    (void)b;
    (void)njobs;
}

void batch_solve_impl(ssmap_batch *b, const void *const *dM, const double *lambda,
                      const ssmap_steps *steps, int iters, void *const *dF, hipStream_t s) {
    const int nj = (int)b->jobs.size();
    bool tune = false;
    for (int j = 0; j < nj; ++j) {
        if (!dM[j] || !dF[j]) fail(SSMAP_EINVAL, "NULL buffer for job " + std::to_string(j));
        validate_steps(b->jobs[j], lambda[j], &steps[j], iters);
        if (steps[j].stop_tol != 0 ||
            (steps[j].flags & (SSMAP_KEEP_AUX | SSMAP_WARM_START | SSMAP_MONITOR_PRIMAL)))
            fail(SSMAP_EINVAL, "batches take no stopping rule, primal residual, SSMAP_KEEP_AUX or "
                               "warm start");
        tune |= (steps[j].flags & SSMAP_AUTOTUNE) != 0;
    }
    ssmap_batch_stats &S = b->stats;
    std::memset(&S, 0, sizeof(S));
    S.njobs = nj;
    S.iters = iters;
    // ---- prepare every job (coefficients, operand images, projection, z^0 = 0)
    HIPC(&b->arena, hipEventRecord(b->ev[0], s));
    std::vector<Prepared> Ps;
    Ps.reserve(nj);
    for (int j = 0; j < nj; ++j) {
        try {
            Ps.push_back(prepare(b->jobs[j], dM[j], lambda[j], &steps[j], iters, s, false));
        } catch (const Fail &f) {
            throw Fail{f.status, "job " + std::to_string(j) + ": " + f.msg};
        }
        S.voxels += (double)b->jobs[j]->g.N;
    }
    HIPC(&b->arena, hipEventRecord(b->ev[1], s));
    // ---- group the fused jobs into shared-launch classes
    std::vector<BatchClass> classes;
    std::vector<int> solo;
    for (int j = 0; j < nj; ++j) {
        const Plan &pl = Ps[j].pl;
        if (!pl.fused) {
            solo.push_back(j);
            continue;
        }
        const bool planar = b->jobs[j]->g.nz == 1;
        int found = -1;
        for (size_t c = 0; c < classes.size(); ++c)
            if (classes[c].mode == pl.mode && classes[c].RP == pl.RP && classes[c].planar == planar &&
                rank_bucket(classes[c].r) == rank_bucket(pl.r))
                found = (int)c;
        if (found < 0) {
            if (classes.size() >= SSMAP_MAX_CLASSES) {
                solo.push_back(j);
                continue;
            }
            BatchClass C;
            C.mode = pl.mode;
            C.r = pl.r;
            C.RP = pl.RP;
            C.planar = planar;
            classes.push_back(C);
            found = (int)classes.size() - 1;
        }
        BatchClass &C = classes[found];
        C.r = std::max(C.r, pl.r);        // the bucket's K-step count covers every member
        C.jobs.push_back(j);
    }
    // ---- brick shape per class: default, or the fastest candidate when tuning
    std::vector<FusedLaunch> Ls(classes.size());
    auto t_tune = std::chrono::steady_clock::now();
    for (size_t c = 0; c < classes.size(); ++c) {
        BatchClass &C = classes[c];
        Grid g0 = b->jobs[C.jobs[0]]->g;
        std::string key = std::to_string(C.mode) + "/" + std::to_string(C.RP) + "/" +
                          std::to_string(C.r) + "/" + (C.planar ? "p" : "v");
        for (int j : C.jobs) key += "," + std::to_string(j);
        const auto kept = b->tuned.find(key);
        FusedShape best = kept != b->tuned.end() ? kept->second : default_shape(C.mode, g0);
        const auto cands = candidate_shapes(C.mode, C.planar);
        if (tune && cands.size() > 1 && iters > 0) {
            float best_ms = 1e30f;
            for (const FusedShape &sh : cands) {
                FusedLaunch L;
                upload_class(b, (int)c, C, Ps, sh, L, s);
                launch_class(b, L, C.jobs.size(), 0, s);             // warm-up
                HIPC(&b->arena, hipEventRecord(b->ev[4], s));
                for (int k = 1; k <= 3; ++k) launch_class(b, L, C.jobs.size(), k, s);
                HIPC(&b->arena, hipEventRecord(b->ev[5], s));
                HIPC(&b->arena, hipEventSynchronize(b->ev[5]));
                const float ms = (float)elapsed_ms(b->ev[4], b->ev[5]);
                if (ms < best_ms) {
                    best_ms = ms;
                    best = sh;
                }
            }
            // the search advanced these jobs' states: start them again from z^0
            for (int j : C.jobs) init_state(b->jobs[j], Ps[j], s);
            b->tuned[key] = best;
        }
        C.shape = best;
        upload_class(b, (int)c, C, Ps, best, Ls[c], s);
        C.ntiles = Ls[c].ntiles;
    }
    HIPC(&b->arena, hipStreamSynchronize(s));
    if (tune)
        S.autotune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                                  t_tune).count();
    // single-job launch plans of the solo jobs (unfused, or beyond the class limit)
    std::vector<FusedLaunch> solo_L(solo.size());
    for (size_t i = 0; i < solo.size(); ++i) {
        if (Ps[solo[i]].pl.fused) solo_L[i] = single_launch(b->jobs[solo[i]], Ps[solo[i]], s);
        Ps[solo[i]].ntiles = solo_L[i].ntiles;
    }
    // monitored jobs: the sums of each job after the iteration, into its own stats
    auto monitor = [&](int j, int k) {
        try {
            (void)monitor_step(b->jobs[j], Ps[j], k, s);
        } catch (const Fail &f) {
            throw Fail{f.status, "job " + std::to_string(j) + ": " + f.msg};
        }
    };
    // ---- the shared iteration loop
    HIPC(&b->arena, hipEventRecord(b->ev[2], s));
    for (int k = 0; k < iters; ++k) {
        for (size_t c = 0; c < classes.size(); ++c) {
            bool any = false;
            for (int j : classes[c].jobs) any |= checked_after(Ps[j], k);
            launch_class(b, Ls[c], classes[c].jobs.size(), k, s, any ? classes[c].mon : nullptr);
        }
        for (size_t i = 0; i < solo.size(); ++i) step_job(b->jobs[solo[i]], Ps[solo[i]], &solo_L[i], k, s);
        for (size_t c = 0; c < classes.size(); ++c)
            for (size_t m = 0; m < classes[c].jobs.size(); ++m) {
                const int j = classes[c].jobs[m];
                if (!checked_after(Ps[j], k)) continue;
                Ps[j].monpart = classes[c].mon + classes[c].tile_off[m];
                Ps[j].ntiles = classes[c].tile_cnt[m];
                monitor(j, k);
            }
        for (int j : solo)
            if (checked_after(Ps[j], k)) monitor(j, k);
    }
    HIPC(&b->arena, hipGetLastError());
    HIPC(&b->arena, hipEventRecord(b->ev[3], s));
    for (int j = 0; j < (int)Ps.size(); ++j) {
        try {
            monitor_flush(b->jobs[j], Ps[j], s);
        } catch (const Fail &f) {
            throw Fail{f.status, "job " + std::to_string(j) + ": " + f.msg};
        }
    }
    for (int j = 0; j < nj; ++j) finish(b->jobs[j], Ps[j], dF[j], s);
    HIPC(&b->arena, hipEventRecord(b->ev[4], s));
    HIPC(&b->arena, hipStreamSynchronize(s));
    S.project_ms = elapsed_ms(b->ev[0], b->ev[1]);
    S.iterate_ms = elapsed_ms(b->ev[2], b->ev[3]);
    S.output_ms = elapsed_ms(b->ev[3], b->ev[4]);
    S.nclasses = (int)classes.size();
    S.solo_jobs = (int)solo.size();
    for (size_t c = 0; c < classes.size(); ++c) {
        S.class_precision[c] = classes[c].mode;
        S.class_rank_padded[c] = classes[c].RP;
        S.class_jobs[c] = (int)classes[c].jobs.size();
        S.class_bricks[c] = classes[c].ntiles;
        S.class_brick_y[c] = classes[c].shape.ty;
        S.class_brick_z[c] = classes[c].shape.tz;
    }
}

template <typename Fn>
ssmap_status batch_guarded(ssmap_batch *b, Fn &&fn) {
    try {
        if (b->poisoned || b->arena.poisoned) fail(SSMAP_EDEVICE, "batch poisoned by an earlier device error");
        for (ssmap_ctx *c : b->jobs)
            if (c->poisoned) fail(SSMAP_EDEVICE, "batch poisoned by an earlier device error");
        fn();
        return SSMAP_OK;
    } catch (const Fail &f) {
        b->err = f.msg;
        if (f.status == SSMAP_EDEVICE) b->poisoned = true;
        return f.status;
    } catch (const std::bad_alloc &) {
        b->err = "host allocation failed";
        return SSMAP_ENOMEM;
    } catch (...) {
        b->err = "unexpected internal error";
        b->poisoned = true;
        return SSMAP_EDEVICE;
    }
}

void free_batch(ssmap_batch *b) {
    if (!b) return;
    for (ssmap_ctx *c : b->jobs) free_ctx(c);
    for (auto &kv : b->arena.bufs) (void)hipFree(kv.second.first);
    b->arena.bufs.clear();
    for (auto &e : b->ev)
        if (e) (void)hipEventDestroy(e);
    delete b;
}

}  // namespace

extern "C" {

const char *ssmap_version(void) { return "ssmap 0.1 (gfx950)"; }

ssmap_status ssmap_create(const double *K, int P, int Q, const int64_t grid[3], ssmap_ctx **out) {
    if (out) *out = nullptr;
    ssmap_ctx *c = nullptr;
    ssmap_status st = guarded(nullptr, [&] {
        if (!K || !grid || !out) fail(SSMAP_EINVAL, "NULL argument");
        if (P < 1 || Q < 1) fail(SSMAP_EINVAL, "P and Q must be >= 1");
        for (int i = 0; i < 3; ++i)
            if (grid[i] < 1) fail(SSMAP_EINVAL, "grid dimensions must be >= 1");
        const double Nd = (double)grid[0] * (double)grid[1] * (double)grid[2];
        if (Nd * (double)((Q + QC - 1) / QC * QC) > 9.0e18)
            fail(SSMAP_EINVAL, "grid too large");
        double fro = 0.0;
        for (size_t i = 0; i < (size_t)P * Q; ++i) {
            if (!std::isfinite(K[i])) fail(SSMAP_ENONFINITE, "K holds a NaN or Inf");
            fro += K[i] * K[i];
        }
        if (!(fro > 0)) fail(SSMAP_EINVAL, "K is zero");
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
            (void)hipGetLastError();
            fail(SSMAP_ENODEV, "no HIP device");
        }
        auto t0 = std::chrono::steady_clock::now();
        c = new ssmap_ctx();
        c->P = P;
        c->Q = Q;
        c->kmin = std::min(P, Q);
        c->Qp = (Q + QC - 1) / QC * QC;
        c->nchunk = c->Qp / QC;
        c->g = Grid{grid[0], grid[1], grid[2], grid[0] * grid[1] * grid[2]};
        if (hipGetDevice(&c->device) != hipSuccess) fail(SSMAP_ENODEV, "hipGetDevice failed");
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, c->device) != hipSuccess)
            fail(SSMAP_ENODEV, "hipGetDeviceProperties failed");
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            fail(SSMAP_ENODEV, std::string("device is ") + prop.gcnArchName + ", need gfx950");
        thin_svd(K, P, Q, c->U, c->s, c->V);
        c->dtd_norm = dtd_norm_closed(c->g);
        // the device's scratch array for allocation-free solves (looked up once per device)
        c->scratch_err = scratch_device_ptr(&c->scratch);
        if (c->scratch_err != hipSuccess) {
            (void)hipGetLastError();
            c->scratch = nullptr;
        }
        for (auto &e : c->ev) HIPC(c, hipEventCreate(&e));
        HIPC(c, hipHostMalloc((void **)&c->host_stats, ST_COUNT * sizeof(double)));
        auto t1 = std::chrono::steady_clock::now();
        c->stats.setup_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        *out = c;
    });
    if (st != SSMAP_OK) {
        free_ctx(c);
        if (out) *out = nullptr;
    }
    return st;
}

ssmap_status ssmap_solve_device(ssmap_ctx *ctx, const void *dM, double lambda,
                                const ssmap_steps *steps, int iters, void *dF, void *hip_stream) {
    if (!ctx) return SSMAP_EINVAL;
    return guarded(ctx, [&] {
        if (!dM || !dF) fail(SSMAP_EINVAL, "NULL buffer");
        validate_steps(ctx, lambda, steps, iters);
        HIPC(ctx, hipSetDevice(ctx->device));
        const double setup = ctx->stats.setup_ms;
        solve_impl(ctx, dM, lambda, steps, iters, dF, (hipStream_t)hip_stream);
        ctx->stats.setup_ms = setup;
    });
}

ssmap_status ssmap_solve_device_noalloc(ssmap_ctx *ctx, const void *dM, double lambda,
                                        const ssmap_steps *steps, int iters, void *dF,
                                        void *hip_stream) {
    if (!ctx) return SSMAP_EINVAL;
    return guarded(ctx, [&] {
        if (!dM || !dF) fail(SSMAP_EINVAL, "NULL buffer");
        validate_steps(ctx, lambda, steps, iters);
        if (steps->flags & SSMAP_KEEP_AUX)
            fail(SSMAP_EINVAL, "an allocation-free solve keeps no aux output (SSMAP_KEEP_AUX)");
        if (steps->flags & SSMAP_WARM_START)
            fail(SSMAP_EINVAL, "an allocation-free solve takes no warm start");
        if (steps->kernel == SSMAP_KERNEL_GEMM)
            fail(SSMAP_EINVAL, "an allocation-free solve runs the fused or unfused kernels");
        HIPC(ctx, hipSetDevice(ctx->device));
        if (!ctx->scratch)
            fail(SSMAP_EDEVICE, std::string("scratch array lookup failed: ") +
                                    hipGetErrorString(ctx->scratch_err));
        // AUTO as in ssmap_solve_device, except that where it would take the GEMM
        // path (its own layouts) the unfused kernels run
        ssmap_steps st = *steps;
        if (st.kernel == SSMAP_KERNEL_AUTO) {
            const int r = rank_rule(ctx->s, st.rank);
            if (!fused_supported(st.precision, (r + 15) / 16 * 16, ctx->g.N))
                st.kernel = SSMAP_KERNEL_UNFUSED;
        }
        struct On {
            ssmap_ctx *c;
            explicit On(ssmap_ctx *c_) : c(c_) {
                c->arena.on = true;
                c->arena.base = (char *)c->scratch;
                c->arena.cap = kScratchBytes;
                c->arena.used = 0;
                c->arena.bufs.clear();
            }
            ~On() {
                c->arena.on = false;
                c->arena.bufs.clear();
            }
        } on(ctx);
        const double setup = ctx->stats.setup_ms;
        solve_impl(ctx, dM, lambda, &st, iters, dF, (hipStream_t)hip_stream);
        ctx->stats.setup_ms = setup;
    });
}

ssmap_status ssmap_solve(ssmap_ctx *ctx, const double *M, double lambda, const ssmap_steps *steps,
                         int iters, double *F_out) {
    if (!ctx) return SSMAP_EINVAL;
    return guarded(ctx, [&] {
        if (!M || !F_out) fail(SSMAP_EINVAL, "NULL buffer");
        validate_steps(ctx, lambda, steps, iters);
        HIPC(ctx, hipSetDevice(ctx->device));
        const int64_t N = ctx->g.N;
        const size_t nm = (size_t)N * ctx->P, nf = (size_t)N * ctx->Q;
        for (size_t i = 0; i < nm; ++i)    // rows outside a mask are not read
            if (!std::isfinite(M[i]) && (ctx->code.empty() || (ctx->code[i / ctx->P] & 0x80)))
                fail(SSMAP_ENONFINITE, "M holds a NaN or Inf");
        const bool f64 = steps->precision == SSMAP_FP64;
        const size_t esz = f64 ? 8 : 4;
        plan_check(ctx, {{"io_M", nm * esz}, {"io_F", nf * esz}});
        void *dM = ensure(ctx, "io_M", nm * esz);
        void *dF = ensure(ctx, "io_F", nf * esz);
        hipStream_t s = nullptr;
        if (f64) {
            HIPC(ctx, hipMemcpy(dM, M, nm * 8, hipMemcpyHostToDevice));
        } else {
            std::vector<float> tmp(M, M + nm);
            HIPC(ctx, hipMemcpy(dM, tmp.data(), nm * 4, hipMemcpyHostToDevice));
        }
        const double setup = ctx->stats.setup_ms;
        solve_impl(ctx, dM, lambda, steps, iters, dF, s);
        ctx->stats.setup_ms = setup;
        if (f64) {
            HIPC(ctx, hipMemcpy(F_out, dF, nf * 8, hipMemcpyDeviceToHost));
        } else {
            std::vector<float> tmp(nf);
            HIPC(ctx, hipMemcpy(tmp.data(), dF, nf * 4, hipMemcpyDeviceToHost));
            for (size_t i = 0; i < nf; ++i) F_out[i] = tmp[i];
        }
    });
}

ssmap_status ssmap_set_mask(ssmap_ctx *ctx, const uint8_t *mask) {
    if (!ctx) return SSMAP_EINVAL;
    return guarded(ctx, [&] {
        HIPC(ctx, hipSetDevice(ctx->device));
        if (!mask) {
            ctx->code.clear();
            ctx->inside = ctx->g.N;
            ctx->dtd_norm = dtd_norm_closed(ctx->g);
            return;
        }
        std::vector<uint8_t> code;
        int64_t inside = 0;
        mask_codes(ctx->g, mask, code, inside);
        void *d = ensure(ctx, "code", code.size());
        HIPC(ctx, hipMemcpy(d, code.data(), code.size(), hipMemcpyHostToDevice));
        ctx->dtd_norm = masked_dtd_norm(ctx->g, code);
        ctx->code.swap(code);
        ctx->inside = inside;
    });
}

ssmap_status ssmap_set_reference(ssmap_ctx *ctx, const double *f_star) {
    if (!ctx) return SSMAP_EINVAL;
    return guarded(ctx, [&] {
        HIPC(ctx, hipSetDevice(ctx->device));
        if (!f_star) {
            ctx->has_ref = false;
            return;
        }
        const size_t n = (size_t)ctx->g.N * ctx->Q;
        double ss = 0.0;
        for (size_t i = 0; i < n; ++i) {
            if (!std::isfinite(f_star[i])) fail(SSMAP_ENONFINITE, "f_star holds a NaN or Inf");
            ss += f_star[i] * f_star[i];
        }
        if (!(ss > 0)) fail(SSMAP_EINVAL, "f_star is zero");
        void *d = ensure(ctx, "fstar", n * 8);
        HIPC(ctx, hipMemcpy(d, f_star, n * 8, hipMemcpyHostToDevice));
        ctx->has_ref = true;
    });
}

ssmap_status ssmap_set_initial(ssmap_ctx *ctx, const double *z0, const double *d0) {
    if (!ctx) return SSMAP_EINVAL;
    return guarded(ctx, [&] {
        HIPC(ctx, hipSetDevice(ctx->device));
        ctx->has_init = false;
        if (!z0 && !d0) {
            ctx->init_z = ctx->init_d = false;
            return;
        }
        const size_t n = (size_t)ctx->g.N * ctx->Q;
        for (const double *p : {z0, d0})
            if (p)
                for (size_t i = 0; i < n; ++i)
                    if (!std::isfinite(p[i])) fail(SSMAP_ENONFINITE, "z0 or d0 holds a NaN or Inf");
        if (z0) HIPC(ctx, hipMemcpy(ensure(ctx, "init_z", n * 8), z0, n * 8, hipMemcpyHostToDevice));
        if (d0) HIPC(ctx, hipMemcpy(ensure(ctx, "init_d", n * 8), d0, n * 8, hipMemcpyHostToDevice));
        ctx->init_z = z0 != nullptr;
        ctx->init_d = d0 != nullptr;
        ctx->has_init = true;
    });
}

ssmap_status ssmap_tune_beta(ssmap_ctx *ctx, const double *M, double lambda,
                             const ssmap_steps *steps, int iters, const double *betas,
                             int n_betas, double *J_out, double *beta_out) {
    if (!ctx) return SSMAP_EINVAL;
    ssmap_ctx *pc = nullptr;
    const ssmap_status st = guarded(ctx, [&] {
        if (!M || !steps || !betas || !beta_out) fail(SSMAP_EINVAL, "NULL argument");
        if (n_betas < 1 || iters < 1) fail(SSMAP_EINVAL, "need n_betas >= 1 and iters >= 1");
        for (int i = 0; i < n_betas; ++i)
            if (!(std::isfinite(betas[i]) && betas[i] > 0)) fail(SSMAP_EINVAL, "candidate beta <= 0");
        ssmap_steps ps = *steps;
        ps.beta = betas[0];
        ps.check_every = iters;          // one float64 objective after the last iteration
        ps.flags = 0;
        ps.stop_tol = 0.0;
        validate_steps(ctx, lambda, &ps, iters);
        HIPC(ctx, hipSetDevice(ctx->device));
        // the centre patch: 3 voxels per axis (fewer on shorter axes)
        const int64_t dims[3] = {ctx->g.nx, ctx->g.ny, ctx->g.nz};
        int64_t org[3], pd[3];
        for (int a = 0; a < 3; ++a) {
            pd[a] = std::min<int64_t>(3, dims[a]);
            org[a] = (dims[a] - pd[a]) / 2;
        }
        const int64_t Np = pd[0] * pd[1] * pd[2];
        std::vector<double> Mp((size_t)Np * ctx->P);
        for (int64_t z = 0; z < pd[2]; ++z)
            for (int64_t y = 0; y < pd[1]; ++y)
                for (int64_t x = 0; x < pd[0]; ++x) {
                    const int64_t src = (org[0] + x) + dims[0] * ((org[1] + y) + dims[1] * (org[2] + z));
                    const int64_t dst = x + pd[0] * (y + pd[1] * z);
                    std::memcpy(&Mp[(size_t)dst * ctx->P], &M[(size_t)src * ctx->P],
                                (size_t)ctx->P * sizeof(double));
                }
        // a context for the patch sharing the dictionary's factors (no new SVD)
        pc = new ssmap_ctx();
        pc->P = ctx->P;
        pc->Q = ctx->Q;
        pc->kmin = ctx->kmin;
        pc->Qp = ctx->Qp;
        pc->nchunk = ctx->nchunk;
        pc->g = Grid{pd[0], pd[1], pd[2], Np};
        pc->device = ctx->device;
        pc->U = ctx->U;
        pc->s = ctx->s;
        pc->V = ctx->V;
        pc->dtd_norm = dtd_norm_closed(pc->g);
        for (auto &e : pc->ev) HIPC(ctx, hipEventCreate(&e));
        HIPC(ctx, hipHostMalloc((void **)&pc->host_stats, ST_COUNT * sizeof(double)));
        std::vector<double> F((size_t)Np * ctx->Q);
        int best = 0;
        std::vector<double> J(n_betas);
        for (int i = 0; i < n_betas; ++i) {
            ps.beta = betas[i];
            if (ssmap_solve(pc, Mp.data(), lambda, &ps, iters, F.data()) != SSMAP_OK)
                fail(pc->poisoned ? SSMAP_EDEVICE : SSMAP_EINVAL, "patch solve failed: " + pc->err);
            J[i] = pc->stats.hist_objective[pc->stats.n_hist - 1];
            if (J[i] < J[best]) best = i;
        }
        if (J_out) std::copy(J.begin(), J.end(), J_out);
        *beta_out = betas[best];
    });
    free_ctx(pc);
    return st;
}

ssmap_status ssmap_get_aux(ssmap_ctx *ctx, double *f_out, double *d_out) {
    if (!ctx) return SSMAP_EINVAL;
    return guarded(ctx, [&] {
        if (!ctx->aux_valid) fail(SSMAP_EINVAL, "no solve with SSMAP_KEEP_AUX has run");
        const int64_t N = ctx->g.N;
        const size_t nf = (size_t)N * ctx->Q;
        double *tmp = (double *)ensure(ctx, "io_aux", nf * 8);
        void *src[2] = {ctx->aux_f, ctx->aux_d};
        double *dst[2] = {f_out, d_out};
        for (int k = 0; k < 2; ++k) {
            if (!dst[k]) continue;
            if (ctx->aux_iters == 0) {
                std::memset(dst[k], 0, nf * 8);
                continue;
            }
            if (ctx->aux_ld > 0)       // GEMM path: voxel-major float32 rows of aux_ld
                launch_gemm_output((const float *)src[k], tmp, true, N, ctx->Q, ctx->aux_ld, nullptr);
            else
                launch_output(ctx->aux_mode, src[k], tmp, ctx->Q, N, true, nullptr);
            HIPC(ctx, hipGetLastError());
            HIPC(ctx, hipMemcpy(dst[k], tmp, nf * 8, hipMemcpyDeviceToHost));
        }
    });
}

ssmap_status ssmap_get_stats(const ssmap_ctx *ctx, ssmap_stats *out) {
    if (!ctx || !out) return SSMAP_EINVAL;
    *out = ctx->stats;
    return SSMAP_OK;
}

ssmap_status ssmap_get_singular_values(const ssmap_ctx *ctx, double *sigma_out, int cap,
                                       int *n_out) {
    if (!ctx || !n_out) return SSMAP_EINVAL;
    *n_out = ctx->kmin;
    if (sigma_out)
        for (int i = 0; i < std::min(cap, ctx->kmin); ++i) sigma_out[i] = ctx->s[i];
    return SSMAP_OK;
}

const char *ssmap_last_error(const ssmap_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

void ssmap_destroy(ssmap_ctx *ctx) { free_ctx(ctx); }

ssmap_status ssmap_batch_create(int njobs, const double *const *K, const int *P, const int *Q,
                                const int64_t *grids, ssmap_batch **out) {
    if (out) *out = nullptr;
    if (njobs < 1 || !K || !P || !Q || !grids || !out) {
        g_batch_create_error = "invalid arguments";
        return SSMAP_EINVAL;
    }
    ssmap_batch *b = nullptr;
    try {
        b = new ssmap_batch();
    } catch (...) {
        g_batch_create_error = "host allocation failed";
        return SSMAP_ENOMEM;
    }
    for (int j = 0; j < njobs; ++j) {
        ssmap_ctx *c = nullptr;
        const ssmap_status st = ssmap_create(K[j], P[j], Q[j], grids + 3 * j, &c);
        if (st != SSMAP_OK) {
            g_batch_create_error = "job " + std::to_string(j) + ": " + g_create_error;
            free_batch(b);
            return st;
        }
        b->jobs.push_back(c);
    }
    for (auto &e : b->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            g_batch_create_error = "hipEventCreate failed";
            free_batch(b);
            return SSMAP_EDEVICE;
        }
    b->stats.njobs = njobs;
    *out = b;
    return SSMAP_OK;
}

ssmap_status ssmap_batch_solve_device(ssmap_batch *b, const void *const *dM, const double *lambda,
                                      const ssmap_steps *steps, int iters, void *const *dF,
                                      void *hip_stream) {
    if (!b) return SSMAP_EINVAL;
    return batch_guarded(b, [&] {
        if (!dM || !lambda || !steps || !dF) fail(SSMAP_EINVAL, "NULL argument");
        HIPC(&b->arena, hipSetDevice(b->jobs[0]->device));
        batch_solve_impl(b, dM, lambda, steps, iters, dF, (hipStream_t)hip_stream);
    });
}

ssmap_status ssmap_batch_get_job_stats(const ssmap_batch *b, int job, ssmap_stats *out) {
    if (!b || !out || job < 0 || job >= (int)b->jobs.size()) return SSMAP_EINVAL;
    *out = b->jobs[job]->stats;
    return SSMAP_OK;
}

ssmap_status ssmap_batch_set_mask(ssmap_batch *b, int job, const uint8_t *mask) {
    if (!b) return SSMAP_EINVAL;
    return batch_guarded(b, [&] {
        if (job < 0 || job >= (int)b->jobs.size()) fail(SSMAP_EINVAL, "job index out of range");
        const ssmap_status st = ssmap_set_mask(b->jobs[job], mask);
        if (st != SSMAP_OK) fail(st, "job " + std::to_string(job) + ": " + ssmap_last_error(b->jobs[job]));
    });
}

ssmap_status ssmap_batch_solve(ssmap_batch *b, const double *const *M, const double *lambda,
                               const ssmap_steps *steps, int iters, double *const *F_out) {
    if (!b) return SSMAP_EINVAL;
    return batch_guarded(b, [&] {
        if (!M || !lambda || !steps || !F_out) fail(SSMAP_EINVAL, "NULL argument");
        const int nj = (int)b->jobs.size();
        HIPC(&b->arena, hipSetDevice(b->jobs[0]->device));
        std::vector<const void *> dM(nj);
        std::vector<void *> dF(nj);
        for (int j = 0; j < nj; ++j) {
            ssmap_ctx *c = b->jobs[j];
            if (!M[j] || !F_out[j]) fail(SSMAP_EINVAL, "NULL buffer for job " + std::to_string(j));
            const size_t nm = (size_t)c->g.N * c->P, nf = (size_t)c->g.N * c->Q;
            for (size_t i = 0; i < nm; ++i)    // rows outside a job's mask are not read
                if (!std::isfinite(M[j][i]) && (c->code.empty() || (c->code[i / c->P] & 0x80)))
                    fail(SSMAP_ENONFINITE, "job " + std::to_string(j) + ": M holds a NaN or Inf");
            const bool f64 = steps[j].precision == SSMAP_FP64;
            const size_t esz = f64 ? 8 : 4;
            void *m = ensure(c, "io_M", nm * esz);
            dF[j] = ensure(c, "io_F", nf * esz);
            if (f64) {
                HIPC(c, hipMemcpy(m, M[j], nm * 8, hipMemcpyHostToDevice));
            } else {
                std::vector<float> tmp(M[j], M[j] + nm);
                HIPC(c, hipMemcpy(m, tmp.data(), nm * 4, hipMemcpyHostToDevice));
            }
            dM[j] = m;
        }
        batch_solve_impl(b, dM.data(), lambda, steps, iters, dF.data(), nullptr);
        for (int j = 0; j < nj; ++j) {
            ssmap_ctx *c = b->jobs[j];
            const size_t nf = (size_t)c->g.N * c->Q;
            if (steps[j].precision == SSMAP_FP64) {
                HIPC(c, hipMemcpy(F_out[j], dF[j], nf * 8, hipMemcpyDeviceToHost));
            } else {
                std::vector<float> tmp(nf);
                HIPC(c, hipMemcpy(tmp.data(), dF[j], nf * 4, hipMemcpyDeviceToHost));
                for (size_t i = 0; i < nf; ++i) F_out[j][i] = tmp[i];
            }
        }
    });
}

ssmap_status ssmap_batch_get_stats(const ssmap_batch *b, ssmap_batch_stats *out) {
    if (!b || !out) return SSMAP_EINVAL;
    *out = b->stats;
    return SSMAP_OK;
}

const char *ssmap_batch_last_error(const ssmap_batch *b) {
    return b ? b->err.c_str() : g_batch_create_error.c_str();
}

void ssmap_batch_destroy(ssmap_batch *b) { free_batch(b); }

}  // extern "C"
