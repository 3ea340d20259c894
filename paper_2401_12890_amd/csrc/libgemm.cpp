// Library products for the exact-rank path: hipBLASLt GEMMs with float32
// accumulation. The path's two contractions (u = V_r w and y = V_r^T z of
// Eq. DictVecSVD, all voxels at once) are plain products C = B A^T of a
// constant M x K operand A and the voxels' N x K operand B, both row-major with
// k contiguous; in hipBLASLt's column-major terms C (M x N) = op(A) op(B) with
// op(A) = A^T (A stored K x M) and op(B) = B (stored K x N). Each distinct shape
// gets its matmul descriptor, layouts and up to kCandidates of the library's
// heuristic algorithms once; the first product of a shape times each candidate
// on the caller's stream in two rounds (one warm-up, then three timed runs per
// round; a candidate's time is its better round, which takes out the first
// runs' clock and cache effects and the order of the candidates) and keeps the
// library's first choice unless another is more than 2 % faster. The choice is
// kept for the life of the process, per device and shape, and every later
// context takes it without timing, so that all solves of a shape in a process
// use one algorithm (one summation order) and give identical results, whichever
// context runs them (a batch job and the same problem solved alone). The
// workspace is allocated once per context.
#include "internal.h"

#include <hip/hip_runtime_api.h>
#include <hipblaslt/hipblaslt.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

namespace ssmap {

struct LibGemm {
    hipblasLtHandle_t h = nullptr;
    void *ws = nullptr;
    size_t wsz = 0;
    struct Plan {
        bool bf16 = false;
        int M = 0, K = 0;
        int64_t N = 0;
        bool ok = false;
        hipblasLtMatmulDesc_t md = nullptr;
        hipblasLtMatrixLayout_t la = nullptr, lb = nullptr, lc = nullptr;
        hipblasLtMatmulAlgo_t algo{};
        std::vector<hipblasLtMatmulAlgo_t> cands;
        bool tuned = false;
    };
    std::vector<Plan> plans;
};

namespace {

constexpr size_t kWorkspace = (size_t)64 << 20;
constexpr int kCandidates = 8;

// The process's choices: (device, bf16, M, N, K) -> index into the heuristic's
// candidate list (the same list for the same shape on the same device).
using ChoiceKey = std::tuple<int, bool, int, int64_t, int>;
std::mutex g_choice_mu;
std::map<ChoiceKey, size_t> g_choice;

bool chosen(const ChoiceKey &k, size_t &idx) {
    std::lock_guard<std::mutex> lk(g_choice_mu);
    auto it = g_choice.find(k);
    if (it == g_choice.end()) return false;
    idx = it->second;
    return true;
}

LibGemm::Plan *plan_for(LibGemm *g, bool bf16, int M, int64_t N, int K) {
    for (auto &p : g->plans)
        if (p.bf16 == bf16 && p.M == M && p.N == N && p.K == K) return &p;
    LibGemm::Plan p;
    p.bf16 = bf16;
    p.M = M;
    p.N = N;
    p.K = K;
    const hipDataType ab = bf16 ? HIP_R_16BF : HIP_R_32F;
    const hipblasOperation_t ta = HIPBLAS_OP_T, tb = HIPBLAS_OP_N;
    hipblasLtMatmulPreference_t pref = nullptr;
    bool ok = hipblasLtMatmulDescCreate(&p.md, HIPBLAS_COMPUTE_32F, HIP_R_32F) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatmulDescSetAttribute(p.md, HIPBLASLT_MATMUL_DESC_TRANSA, &ta, sizeof(ta)) ==
                  HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatmulDescSetAttribute(p.md, HIPBLASLT_MATMUL_DESC_TRANSB, &tb, sizeof(tb)) ==
                  HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatrixLayoutCreate(&p.la, ab, K, M, K) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatrixLayoutCreate(&p.lb, ab, K, N, K) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatrixLayoutCreate(&p.lc, HIP_R_32F, M, N, M) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatmulPreferenceCreate(&pref) == HIPBLAS_STATUS_SUCCESS;
    size_t wsz = kWorkspace;
    if (ok)
        ok = hipblasLtMatmulPreferenceSetAttribute(pref, HIPBLASLT_MATMUL_PREF_MAX_WORKSPACE_BYTES, &wsz,
                                                   sizeof(wsz)) == HIPBLAS_STATUS_SUCCESS;
    if (ok) {
        hipblasLtMatmulHeuristicResult_t heur[kCandidates];
        int n = 0;
        ok = hipblasLtMatmulAlgoGetHeuristic(g->h, p.md, p.la, p.lb, p.lc, p.lc, pref, kCandidates, heur,
                                             &n) == HIPBLAS_STATUS_SUCCESS;
        for (int i = 0; ok && i < n; ++i)
            if (heur[i].state == HIPBLAS_STATUS_SUCCESS && heur[i].workspaceSize <= kWorkspace)
                p.cands.push_back(heur[i].algo);
        ok = ok && !p.cands.empty();
        if (ok) p.algo = p.cands[0];
    }
    if (pref) (void)hipblasLtMatmulPreferenceDestroy(pref);
    p.ok = ok;
    g->plans.push_back(p);
    return &g->plans.back();
}

}  // namespace

LibGemm *libgemm_create() {
    LibGemm *g = new LibGemm();
    if (hipblasLtCreate(&g->h) != HIPBLAS_STATUS_SUCCESS) {
        delete g;
        return nullptr;
    }
    if (hipMalloc(&g->ws, kWorkspace) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipblasLtDestroy(g->h);
        delete g;
        return nullptr;
    }
    g->wsz = kWorkspace;
    return g;
}

void libgemm_destroy(LibGemm *g) {
    if (!g) return;
    for (auto &p : g->plans) {
        if (p.la) (void)hipblasLtMatrixLayoutDestroy(p.la);
        if (p.lb) (void)hipblasLtMatrixLayoutDestroy(p.lb);
        if (p.lc) (void)hipblasLtMatrixLayoutDestroy(p.lc);
        if (p.md) (void)hipblasLtMatmulDescDestroy(p.md);
    }
    if (g->ws) (void)hipFree(g->ws);
    if (g->h) (void)hipblasLtDestroy(g->h);
    delete g;
}

bool libgemm_tn(LibGemm *g, bool bf16, const void *A, const void *B, float *C, int M, int64_t N, int K,
                hipStream_t s) {
    if (!g) return false;
    LibGemm::Plan *p = plan_for(g, bf16, M, N, K);
    if (!p->ok) return false;
    if (!A) return true;                 // shape check only
    const float alpha = 1.0f, beta = 0.0f;
    auto run = [&](const hipblasLtMatmulAlgo_t &algo) {
        return hipblasLtMatmul(g->h, p->md, &alpha, A, p->la, B, p->lb, &beta, C, p->lc, C, p->lc, &algo,
                               g->ws, g->wsz, s) == HIPBLAS_STATUS_SUCCESS;
    };
    if (!p->tuned) {
        p->tuned = true;
        int dev = 0;
        (void)hipGetDevice(&dev);
        const ChoiceKey key{dev, bf16, M, N, K};
        size_t idx = 0;
        if (chosen(key, idx) && idx < p->cands.size()) {
            p->algo = p->cands[idx];
        } else if (p->cands.size() > 1) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
                const size_t nc = p->cands.size();
                std::vector<float> t(nc, -1.0f);
                for (int round = 0; round < 2; ++round)
                    for (size_t i = 0; i < nc; ++i) {
                        const auto &algo = p->cands[i];
                        float ms = 0.0f;
                        if ((round == 0 && !run(algo)) || hipEventRecord(e0, s) != hipSuccess || !run(algo) ||
                            !run(algo) || !run(algo) || hipEventRecord(e1, s) != hipSuccess ||
                            hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                            (void)hipGetLastError();
                            continue;
                        }
                        if (t[i] < 0.0f || ms < t[i]) t[i] = ms;
                    }
                size_t bi = 0;
                for (size_t i = 1; i < nc; ++i)
                    if (t[i] > 0.0f && (t[bi] < 0.0f || t[i] < t[bi])) bi = i;
                idx = (t[0] > 0.0f && t[bi] > 0.98f * t[0]) ? 0 : bi;
                std::lock_guard<std::mutex> lk(g_choice_mu);
                idx = g_choice.emplace(key, idx).first->second;   // a choice made meanwhile wins
                p->algo = p->cands[idx < p->cands.size() ? idx : 0];
            }
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    }
    return run(p->algo);
}

}  // namespace ssmap
