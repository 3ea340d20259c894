// Exact-rank iteration (r above the fused kernels' 32): the two contractions
// of the reduced form (u = V_r w, y = V_r^T z; Eq. DictVecSVD) are dense
// matrix products over all voxels, run as MFMA-tiled GEMMs, with the stencil /
// projected z-update (Eq. z2) and the r-vector recursion as separate
// elementwise passes.
//
// Layouts (voxel-major, padded): z, u: N x Qg; w, y, a.h: N x Rg (Qg, Rg
// multiples of 128, padding 0). bf16x3 keeps the hi/lo/hi bf16 split of each
// voxel's w (3 Rg values) and z (3 Qg values) so that one bf16 product over a
// tripled K gives hi*hi + lo*hi + hi*lo with float32 accumulation.
//
// GEMM: C[n][m] = sum_k A[m][k] B[n][k] (A: M x K row-major, B: N x K
// row-major, C: N x M row-major), M and K multiples of the tiles, N ragged.
// All operands have k contiguous, so a lane's MFMA fragment is one 16-byte read.
#include "internal.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ssmap {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

constexpr int GNT = 256;       // threads: 4 waves in a 2 x 2 arrangement

// K per staged tile and LDS row length (elements) of each operand type.
template <typename T> struct GK;
template <> struct GK<float> {
    static constexpr int KT = 16;
    static constexpr int LD = KT + 1;          // rows 17 floats apart: conflict-free reads
};
template <> struct GK<uint16_t> {
    static constexpr int KT = 64;
    static constexpr int LD = KT + 8;          // rows 144 B apart
};

// Workgroup tile (2 TM x 16) x (2 TN x 16): each wave owns TM x TN MFMA tiles of
// 16 x 16. Larger wave tiles read fewer LDS bytes per product (the bf16 kernel
// needs 8 x 4 to stay within the LDS bandwidth at the matrix-core rate).
template <typename T, int TM, int TN>
__global__ void __launch_bounds__(GNT, 2)
k_gemm_tn(const T *__restrict__ A, const T *__restrict__ B, float *__restrict__ C, int M, int K,
          int64_t N) {
    using G = GK<T>;
    constexpr int KT = G::KT, LD = G::LD;
    constexpr int BM = 32 * TM, BN = 32 * TN;         // workgroup tile
    constexpr int EPV = 16 / (int)sizeof(T);          // elements per 16-byte vector
    constexpr int VPR = KT / EPV;                     // vectors per tile row
    constexpr int NVA = BM * VPR / GNT, NVB = BN * VPR / GNT;   // vectors per thread
    static_assert(NVA >= 1 && NVB >= 1 && BM * VPR % GNT == 0 && BN * VPR % GNT == 0,
                  "tile staging must split over the threads");
    __shared__ __attribute__((aligned(16))) T As[BM * LD];
    __shared__ __attribute__((aligned(16))) T Bs[BN * LD];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 16 * TM, wn = (wave >> 1) * 16 * TN;
    const int m0 = blockIdx.y * BM;
    const int64_t n0 = (int64_t)blockIdx.x * BN;

    // staging: thread -> (row, vector) of the BM x KT and BN x KT tiles (rows of B beyond N load 0)
    v4u ra[NVA], rb[NVB];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int v = 0; v < NVA; ++v) {
            const int e = tid + GNT * v, row = e / VPR, vec = e % VPR;
            ra[v] = *(const v4u *)(A + (size_t)(m0 + row) * K + k0 + vec * EPV);
        }
#pragma unroll
        for (int v = 0; v < NVB; ++v) {
            const int e = tid + GNT * v, row = e / VPR, vec = e % VPR;
            const int64_t n = n0 + row;
            rb[v] = n < N ? *(const v4u *)(B + (size_t)n * K + k0 + vec * EPV) : v4u{0, 0, 0, 0};
        }
    };
    auto put = [&](T *dst, const v4u &v) {
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int i = 0; i < 4; ++i) ((float *)dst)[i] = __uint_as_float(v[i]);
        } else {
            *(v4u *)dst = v;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int v = 0; v < NVA; ++v) {
            const int e = tid + GNT * v;
            put(As + (e / VPR) * LD + (e % VPR) * EPV, ra[v]);
        }
#pragma unroll
        for (int v = 0; v < NVB; ++v) {
            const int e = tid + GNT * v;
            put(Bs + (e / VPR) * LD + (e % VPR) * EPV, rb[v]);
        }
    };

    v4f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0, 0, 0, 0};

    const int r16 = lane & 15, g4 = lane >> 4;
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += KT) {
        __syncthreads();                  // the previous tile is consumed
        stash();
        __syncthreads();
        if (k0 + KT < K) fetch(k0 + KT);  // next tile in flight during the products
        if constexpr (sizeof(T) == 4) {
            // v_mfma_f32_16x16x4f32: lane holds A[m = l % 16][k = l / 16], B[n = l % 16][k = l / 16]
#pragma unroll
            for (int ks = 0; ks < KT; ks += 4) {
                float a[TM], b[TN];
#pragma unroll
                for (int i = 0; i < TM; ++i) a[i] = ((const float *)As)[(wm + 16 * i + r16) * LD + ks + g4];
#pragma unroll
                for (int j = 0; j < TN; ++j) b[j] = ((const float *)Bs)[(wn + 16 * j + r16) * LD + ks + g4];
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        } else {
            // v_mfma_f32_16x16x32_bf16: lane holds 8 consecutive k (8 (l / 16) .. +7)
#pragma unroll
            for (int ks = 0; ks < KT; ks += 32) {
                v8bf a[TM], b[TN];
#pragma unroll
                for (int i = 0; i < TM; ++i)
                    a[i] = *(const v8bf *)(As + (wm + 16 * i + r16) * LD + ks + 8 * g4);
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    b[j] = *(const v8bf *)(Bs + (wn + 16 * j + r16) * LD + ks + 8 * g4);
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        }
    }
    // D layout: lane holds rows (m) 4 (l / 16) + i of column (n) l % 16: 16 contiguous bytes of C
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int64_t n = n0 + wn + 16 * j + r16;
        if (n >= N) continue;
#pragma unroll
        for (int i = 0; i < TM; ++i)
            *(v4f *)(C + (size_t)n * M + m0 + wm + 16 * i + 4 * g4) = acc[i][j];
    }
}

__device__ __forceinline__ uint16_t bf16_rne_bits(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// hi/lo/hi bf16 split of a float row segment: dst[3 L] = (hi[0..L), lo[0..L), hi[0..L))
__device__ __forceinline__ void split3(float v, uint16_t *dst, int k, int L) {
    const uint16_t h = bf16_rne_bits(v);
    const uint16_t l = bf16_rne_bits(v - __uint_as_float((unsigned)h << 16));
    dst[k] = h;
    dst[L + k] = l;
    dst[2 * L + k] = h;
}

// z^{k+1} = max(0, z - tau (2 lambda (deg z - sum of neighbours) - beta u)) per (voxel, node);
// outside a mask z stays 0. One thread per (voxel, 4 nodes).
__global__ void __launch_bounds__(256)
k_gemm_update(const float *__restrict__ z, const float *__restrict__ u, float *__restrict__ zn,
              uint16_t *__restrict__ zs, Grid g, int Qg, float tau, float lam2, float beta,
              const uint8_t *__restrict__ code) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int q4 = Qg / 4;
    if (idx >= g.N * q4) return;
    const int64_t n = idx / q4;
    const int q = (int)(idx % q4) * 4;
    const int64_t x = n % g.nx, y = (n / g.nx) % g.ny, zz = n / (g.nx * g.ny);
    const size_t o = (size_t)n * Qg + q;
    const v4f zc = *(const v4f *)(z + o);
    v4f nsum = v4f{0, 0, 0, 0};
    int deg = 0;
    const int64_t sy = g.nx, sz = g.nx * g.ny;
    if (x > 0) { nsum += *(const v4f *)(z + o - Qg); ++deg; }
    if (x + 1 < g.nx) { nsum += *(const v4f *)(z + o + Qg); ++deg; }
    if (y > 0) { nsum += *(const v4f *)(z + o - sy * Qg); ++deg; }
    if (y + 1 < g.ny) { nsum += *(const v4f *)(z + o + sy * Qg); ++deg; }
    if (zz > 0) { nsum += *(const v4f *)(z + o - sz * Qg); ++deg; }
    if (zz + 1 < g.nz) { nsum += *(const v4f *)(z + o + sz * Qg); ++deg; }
    bool inside = true;
    if (code) {
        const unsigned cb = code[n];
        inside = (cb & 0x80u) != 0;
        deg = (int)(cb & 7u);
    }
    const v4f uu = *(const v4f *)(u + o);
    v4f r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float lap = (float)deg * zc[i] - nsum[i];
        const float v = zc[i] - tau * (lam2 * lap - beta * uu[i]);
        r[i] = (v > 0.0f && inside) ? v : 0.0f;
    }
    *(v4f *)(zn + o) = r;
    if (zs) {
        uint16_t *d = zs + (size_t)n * 3 * Qg;
#pragma unroll
        for (int i = 0; i < 4; ++i) split3(r[i], d, q + i, Qg);
    }
}

// w^{k+1} = a.h - b.(2 y^{k+1} - y^k - w^k) per (voxel, rank), and its bf16 split.
__global__ void __launch_bounds__(256)
k_gemm_w(const float *__restrict__ ah, const float *__restrict__ ynew, const float *__restrict__ yold,
         float *__restrict__ w, uint16_t *__restrict__ ws, const float *__restrict__ bcoef,
         int64_t N, int Rg) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * Rg) return;
    const int64_t n = idx / Rg;
    const int i = (int)(idx % Rg);
    const float v = ah[idx] - bcoef[i] * (2.0f * ynew[idx] - yold[idx] - w[idx]);
    w[idx] = v;
    if (ws) split3(v, ws + (size_t)n * 3 * Rg, i, Rg);
}

// [i][n] (rank-major, RP rows) -> [n][i] (voxel-major, Rg columns), zero padded;
// optionally the bf16 split of the result.
__global__ void __launch_bounds__(256)
k_gemm_from_ranks(const float *__restrict__ src, int RP, float *__restrict__ dst, uint16_t *__restrict__ ds,
                  int64_t N, int Rg) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * Rg) return;
    const int64_t n = idx / Rg;
    const int i = (int)(idx % Rg);
    const float v = i < RP ? src[(size_t)i * N + n] : 0.0f;
    dst[idx] = v;
    if (ds) split3(v, ds + (size_t)n * 3 * Rg, i, Rg);
}

// z (N x Qg) -> F (N x Q), float32 or float64 output.
template <typename TO>
__global__ void __launch_bounds__(256)
k_gemm_output(const float *__restrict__ z, TO *__restrict__ F, int64_t N, int Q, int Qg) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * Q) return;
    const int64_t n = idx / Q;
    const int q = (int)(idx % Q);
    F[idx] = (TO)z[(size_t)n * Qg + q];
}

inline unsigned nblocks(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }

}  // namespace

bool launch_gemm_tn(bool bf16, const void *A, const void *B, float *C, int M, int K, int64_t N,
                    hipStream_t s) {
    if (M % 128 || K % (bf16 ? GK<uint16_t>::KT : GK<float>::KT) || N <= 0) return false;
    const dim3 block(GNT);
    if (bf16 && M % 256 == 0) {
        // 256 x 128 workgroup tiles, 128 x 64 per wave
        hipLaunchKernelGGL((k_gemm_tn<uint16_t, 8, 4>), dim3(nblocks(N, 128), (unsigned)(M / 256)), block,
                           0, s, (const uint16_t *)A, (const uint16_t *)B, C, M, K, N);
    } else if (bf16) {
        hipLaunchKernelGGL((k_gemm_tn<uint16_t, 4, 4>), dim3(nblocks(N, 128), (unsigned)(M / 128)), block,
                           0, s, (const uint16_t *)A, (const uint16_t *)B, C, M, K, N);
    } else {
        hipLaunchKernelGGL((k_gemm_tn<float, 4, 4>), dim3(nblocks(N, 128), (unsigned)(M / 128)), block, 0,
                           s, (const float *)A, (const float *)B, C, M, K, N);
    }
    return true;
}

void launch_gemm_update(const float *z, const float *u, float *zn, uint16_t *zs, Grid g, int Qg,
                        double tau, double lam2, double beta, const uint8_t *code, hipStream_t s) {
    hipLaunchKernelGGL(k_gemm_update, dim3(nblocks(g.N * (Qg / 4), 256)), dim3(256), 0, s, z, u, zn, zs,
                       g, Qg, (float)tau, (float)lam2, (float)beta, code);
}

void launch_gemm_w(const float *ah, const float *ynew, const float *yold, float *w, uint16_t *ws,
                   const float *bcoef, int64_t N, int Rg, hipStream_t s) {
    hipLaunchKernelGGL(k_gemm_w, dim3(nblocks(N * Rg, 256)), dim3(256), 0, s, ah, ynew, yold, w, ws,
                       bcoef, N, Rg);
}

void launch_gemm_from_ranks(const float *src, int RP, float *dst, uint16_t *ds, int64_t N, int Rg,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_gemm_from_ranks, dim3(nblocks(N * Rg, 256)), dim3(256), 0, s, src, RP, dst, ds,
                       N, Rg);
}

void launch_gemm_output(const float *z, void *F, bool to_double, int64_t N, int Q, int Qg,
                        hipStream_t s) {
    if (to_double)
        hipLaunchKernelGGL(k_gemm_output<double>, dim3(nblocks(N * Q, 256)), dim3(256), 0, s, z,
                           (double *)F, N, Q, Qg);
    else
        hipLaunchKernelGGL(k_gemm_output<float>, dim3(nblocks(N * Q, 256)), dim3(256), 0, s, z,
                           (float *)F, N, Q, Qg);
}

}  // namespace ssmap
