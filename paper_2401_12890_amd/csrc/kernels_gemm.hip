// Exact-rank iteration (r above the fused kernels' 32): the two contractions
// of the reduced form (u = V_r w, y = V_r^T z; Eq. DictVecSVD) are dense
// matrix products over all voxels, run as MFMA-tiled GEMMs whose epilogues
// apply the elementwise steps to the tile in registers: the product u feeds
// the stencil / projected z-update (Eq. z2) and the product y the r-vector
// recursion, so neither u nor y is written to memory.
//
// Layouts (voxel-major, padded): z: N x Qg; w, s, a.h: N x Rg (Qg, Rg
// multiples of 128, padding 0). bf16x3 keeps the hi/lo bf16 split of each
// voxel's w (2 Rg values) and z (2 Qg values); the product runs over a tripled
// K whose third segment reads the hi half again (the constant operand is
// hi | hi | lo), so one bf16 product gives hi*hi + hi*lo + lo*hi with float32
// accumulation.
//
// The r-vector recursion w^{k+1} = a.h - b.(2 y^{k+1} - y^k - w^k) is carried
// with s^k = y^k + w^k in place of the pair (y^k, w^k): w^{k+1} = a.h -
// b.(2 y^{k+1} - s^k), s^{k+1} = y^{k+1} + w^{k+1}, s^0 = w^0 (y^0 = 0).
//
// GEMM: C[n][m] = sum_k A[m][k] B[n][k] (A: M x K row-major; B: N rows of KB
// values, column k of B read at k mod KB), M, K and KB multiples of the tiles,
// N ragged. All operands have k contiguous, so a lane's MFMA fragment is one
// 16-byte read.
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
    static constexpr int LD = KT;              // rows 128 B, 16-byte units swizzled (see sw)
};

__device__ __forceinline__ uint16_t bf16_rne_bits(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// hi/lo bf16 split of a float row segment: dst[2 L] = (hi[0..L), lo[0..L))
__device__ __forceinline__ void split2(float v, uint16_t *dst, int k, int L) {
    const uint16_t h = bf16_rne_bits(v);
    const uint16_t l = bf16_rne_bits(v - __uint_as_float((unsigned)h << 16));
    dst[k] = h;
    dst[L + k] = l;
}

// The same split of 4 consecutive values (k a multiple of 4): two 8-byte stores,
// three with nseg = 3 (hi | lo | hi: the operand of a library product, whose K
// does not wrap).
__device__ __forceinline__ void split2x4(const v4f &v, uint16_t *dst, int k, int L, int nseg = 2) {
    unsigned h[4], l[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        h[i] = bf16_rne_bits(v[i]);
        l[i] = bf16_rne_bits(v[i] - __uint_as_float(h[i] << 16));
    }
    const uint2 hh{h[0] | (h[1] << 16), h[2] | (h[3] << 16)};
    const uint2 ll{l[0] | (l[1] << 16), l[2] | (l[3] << 16)};
    *(uint2 *)(dst + k) = hh;
    *(uint2 *)(dst + L + k) = ll;
    if (nseg == 3) *(uint2 *)(dst + 2 * L + k) = hh;
}

// Epilogue of u = V_r w: z^{k+1} = max(0, z - tau (2 lambda (deg z - sum of
// neighbours) - beta u)) for the voxel's 4 nodes q..q+3; outside a mask z stays 0.
constexpr int EPI_RUN = 4;   // voxels along x per k_epi_z block

struct EpiZ {
    const float *z;
    float *zn;
    uint16_t *zs;            // bf16 split of z^{k+1} (bf16x3) or null
    Grid g;
    int Qg;
    float tau, lam2, beta;
    const uint8_t *code;     // mask codes or null
    int nseg;                // split segments per row: 2 (hi | lo) or 3 (hi | lo | hi)
};

// Per-voxel part of the z-update, shared by the voxel's nodes: the rows of z
// at the voxel and its six face neighbours (a missing neighbour points at the
// voxel's own row and is weighted 0, so every load is unconditional and valid).
struct ColZ {
    const float *c, *nb[6];
    float wt[6];
    float deg;
    bool inside;
    int64_t n;
};

__device__ __forceinline__ ColZ column(const EpiZ &e, int64_t n) {
    const Grid &g = e.g;
    const int64_t x = n % g.nx, t = n / g.nx, y = t % g.ny, zz = t / g.ny;
    const int64_t step[3] = {(int64_t)e.Qg, g.nx * (int64_t)e.Qg, g.nx * g.ny * (int64_t)e.Qg};
    const bool lo[3] = {x > 0, y > 0, zz > 0};
    const bool hi[3] = {x + 1 < g.nx, y + 1 < g.ny, zz + 1 < g.nz};
    ColZ c;
    c.n = n;
    c.c = e.z + n * (int64_t)e.Qg;
    int deg = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c.nb[2 * d] = lo[d] ? c.c - step[d] : c.c;
        c.nb[2 * d + 1] = hi[d] ? c.c + step[d] : c.c;
        c.wt[2 * d] = lo[d] ? 1.0f : 0.0f;
        c.wt[2 * d + 1] = hi[d] ? 1.0f : 0.0f;
        deg += (int)lo[d] + (int)hi[d];
    }
    c.inside = true;
    if (e.code) {
        const unsigned cb = e.code[n];
        c.inside = (cb & 0x80u) != 0;
        deg = (int)(cb & 7u);
    }
    c.deg = (float)deg;
    return c;
}

// The projected z-update of one voxel's nodes q .. q + 3 from z there, its six
// face-neighbour rows (weighted as the column says) and u; stores z^{k+1} and
// its bf16 split.
__device__ __forceinline__ void zupdate(const EpiZ &e, const ColZ &c, int q, const v4f &zc, const v4f (&nb)[6],
                                        const v4f &u) {
    v4f nsum = v4f{0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 6; ++k) nsum += c.wt[k] * nb[k];
    v4f r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float lap = c.deg * zc[i] - nsum[i];
        const float v = zc[i] - e.tau * (e.lam2 * lap - e.beta * u[i]);
        r[i] = (v > 0.0f && c.inside) ? v : 0.0f;
    }
    *(v4f *)(e.zn + c.n * (int64_t)e.Qg + q) = r;
    if (e.zs) split2x4(r, e.zs + c.n * e.nseg * (int64_t)e.Qg, q, e.Qg, e.nseg);
}

// G steps of one voxel (nodes q[g] .. q[g] + 3): every load is issued before any
// result is computed, so a lane has 7 G loads in flight instead of 7 (the
// epilogue is bound by their latency).
template <int G>
__device__ __forceinline__ void epilogue_batch(const EpiZ &e, const ColZ &c, const int (&q)[G],
                                               const v4f (&u)[G]) {
    v4f zc[G], nb[G][6];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        zc[g] = *(const v4f *)(c.c + q[g]);
#pragma unroll
        for (int k = 0; k < 6; ++k) nb[g][k] = *(const v4f *)(c.nb[k] + q[g]);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) zupdate(e, c, q[g], zc[g], nb[g], u[g]);
}

// Epilogue of y = V_r^T z: w^{k+1} = a.h - b.(2 y^{k+1} - s^k), s^{k+1} =
// y^{k+1} + w^{k+1} for the voxel's ranks i..i+3 (s updated in place); w^{k+1}
// goes out as float32 (w) or as its bf16 split (ws).
struct EpiW {
    const float *ah;
    float *s;
    float *w;                // float32 operand of the next u product, or null
    uint16_t *ws;            // its bf16 split (bf16x3), or null
    const float *bcoef;
    int Rg;
    int nseg;                // split segments per row: 2 or 3
};

struct ColW {
    int64_t o;               // first element of the voxel's row
};

__device__ __forceinline__ ColW column(const EpiW &e, int64_t n) { return ColW{n * (int64_t)e.Rg}; }

template <int G>
__device__ __forceinline__ void epilogue_batch(const EpiW &e, const ColW &c, const int (&q)[G],
                                               const v4f (&y)[G]) {
    v4f a[G], sk[G], b[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        a[g] = *(const v4f *)(e.ah + c.o + q[g]);
        sk[g] = *(const v4f *)(e.s + c.o + q[g]);
        b[g] = *(const v4f *)(e.bcoef + q[g]);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        v4f w, s1;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            w[t] = a[g][t] - b[g][t] * (2.0f * y[g][t] - sk[g][t]);
            s1[t] = y[g][t] + w[t];
        }
        *(v4f *)(e.s + c.o + q[g]) = s1;
        if (e.ws) split2x4(w, e.ws + e.nseg * c.o, q[g], e.Rg, e.nseg);
        else *(v4f *)(e.w + c.o + q[g]) = w;
    }
}

// Steps per epilogue batch: GZ for the stencil (7 loaded vectors a step; the
// caller picks it against its register budget), 8 for the r-vectors.
template <typename E, int GZ> struct EpiBatch;
template <int GZ> struct EpiBatch<EpiZ, GZ> { static constexpr int value = GZ; };
template <int GZ> struct EpiBatch<EpiW, GZ> { static constexpr int value = 8; };

// The epilogue of a wave's TM x TN accumulator tiles: lane holds rows (m)
// 4 (l / 16) + i of column (n) l % 16 of each 16 x 16 tile.
template <int TM, int TN, int GZ, typename E>
__device__ __forceinline__ void run_epilogue(const E &epi, const v4f (&acc)[TM][TN], int m0, int64_t n0,
                                             int64_t N, int lane) {
    constexpr int G = EpiBatch<E, GZ>::value < TM ? EpiBatch<E, GZ>::value : TM;
    static_assert(TM % G == 0, "epilogue batches must tile the wave's rows");
    const int r16 = lane & 15, g4 = lane >> 4;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
        const int64_t n = n0 + 16 * j + r16;
        if (n >= N) continue;
        const auto col = column(epi, n);
#pragma unroll
        for (int i0 = 0; i0 < TM; i0 += G) {
            int q[G];
            v4f v[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                q[g] = m0 + 16 * (i0 + g) + 4 * g4;
                v[g] = acc[i0 + g][j];
            }
            epilogue_batch<G>(epi, col, q, v);
        }
    }
}

// Workgroup tile (2 TM x 16) x (2 TN x 16): each wave owns TM x TN MFMA tiles of
// 16 x 16. Larger wave tiles read fewer LDS bytes per product (the bf16 kernel
// needs 8 x 4 to stay within the LDS bandwidth at the matrix-core rate).
template <typename T, int TM, int TN, typename E>
__global__ void __launch_bounds__(GNT, 2)
k_gemm_tn(const T *__restrict__ A, const T *__restrict__ B, int M, int K, int KB, int64_t N, E epi) {
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
    // M blocks fastest: the M / BM tiles that share one block of B rows run at
    // the same time (after the first, their B reads hit the caches), and the
    // grid sweeps the voxels in order, so the z rows one plane away that the
    // stencil epilogue reads are recent enough to be cached. Ordering the
    // tiles per XCD instead measured no better.
    const unsigned t = blockIdx.x;
    const int MB = M / BM;
    const int m0 = (int)(t % MB) * BM;
    const int64_t n0 = (int64_t)(t / MB) * BN;

    // staging: thread -> (row, vector) of the BM x KT and BN x KT tiles (rows of B beyond N load 0)
    v4u ra[NVA], rb[NVB];
    auto fetch = [&](int k0) {
        const int kb = k0 % KB;           // a K tile never straddles a multiple of KB
#pragma unroll
        for (int v = 0; v < NVA; ++v) {
            const int e = tid + GNT * v, row = e / VPR, vec = e % VPR;
            ra[v] = *(const v4u *)(A + (size_t)(m0 + row) * K + k0 + vec * EPV);
        }
#pragma unroll
        for (int v = 0; v < NVB; ++v) {
            const int e = tid + GNT * v, row = e / VPR, vec = e % VPR;
            const int64_t n = n0 + row;
            rb[v] = n < N ? *(const v4u *)(B + (size_t)n * KB + kb + vec * EPV) : v4u{0, 0, 0, 0};
        }
    };
    // 16-byte unit u of LDS row `row`: bf16 rows are unpadded and the unit index
    // is XORed with row % 8, so the fragment reads (16 rows x 4 units) and the
    // staging stores (8 units of consecutive rows) both run at the full LDS rate
    // (measured; padded 144-byte rows cost a third more LDS cycles per read)
    auto sw = [](int row, int u) { return sizeof(T) == 2 ? u ^ (row & 7) : u; };
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
            put(As + (e / VPR) * LD + sw(e / VPR, e % VPR) * EPV, ra[v]);
        }
#pragma unroll
        for (int v = 0; v < NVB; ++v) {
            const int e = tid + GNT * v;
            put(Bs + (e / VPR) * LD + sw(e / VPR, e % VPR) * EPV, rb[v]);
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
                    a[i] = *(const v8bf *)(As + (wm + 16 * i + r16) * LD + sw(r16, ks / 8 + g4) * 8);
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    b[j] = *(const v8bf *)(Bs + (wn + 16 * j + r16) * LD + sw(r16, ks / 8 + g4) * 8);
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        }
    }
    // float32: single stencil steps keep the kernel at four waves per SIMD
    run_epilogue<TM, TN, sizeof(T) == 4 ? 1 : 2>(epi, acc, m0 + wm, n0 + wn, N, lane);
}

// [i][n] (rank-major, RP rows) -> [n][i] (voxel-major, Rg columns), zero padded;
// optionally the bf16 split of the result.
__global__ void __launch_bounds__(256)
k_gemm_from_ranks(const float *__restrict__ src, int RP, float *__restrict__ dst, uint16_t *__restrict__ ds,
                  int64_t N, int Rg, int nseg) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * Rg) return;
    const int64_t n = idx / Rg;
    const int i = (int)(idx % Rg);
    const float v = i < RP ? src[(size_t)i * N + n] : 0.0f;
    dst[idx] = v;
    if (ds) {
        uint16_t *row = ds + (size_t)n * nseg * Rg;
        split2(v, row, i, Rg);
        if (nseg == 3) row[2 * Rg + i] = row[i];
    }
}

// The epilogues on a product that a library GEMM left in memory (voxel-major,
// P[n][m], m over M = Qg or Rg): one lane per voxel and 4 consecutive rows m.
__global__ void __launch_bounds__(256)
k_epi_z(EpiZ e, const float *__restrict__ U) {
    // a block: one tile of 256 node quads for EPI_RUN consecutive voxels n0 ..
    // (the x-neighbours of voxel n are the rows of n - 1 and n + 1, so the run
    // reads EPI_RUN + 2 rows along x instead of 3 EPI_RUN; the y and z
    // neighbours and u per voxel). Every load is issued before any result.
    const int per = e.Qg / 4;
    const int64_t qt = (per + 255) / 256;
    const int64_t n0 = (int64_t)(blockIdx.x / qt) * EPI_RUN;
    const int qi = (int)(blockIdx.x % qt) * 256 + (int)threadIdx.x;
    const int64_t N = e.g.N;
    if (qi >= per || n0 >= N) return;
    const int q = 4 * qi;
    const int64_t Q = e.Qg;
    v4f xr[EPI_RUN + 2];                 // rows n0 - 1 .. n0 + EPI_RUN (clamped to the grid)
#pragma unroll
    for (int j = 0; j < EPI_RUN + 2; ++j) {
        const int64_t n = n0 - 1 + j;
        xr[j] = *(const v4f *)(e.z + (n < 0 ? 0 : n >= N ? N - 1 : n) * Q + q);
    }
    ColZ col[EPI_RUN];
    v4f yz[EPI_RUN][4], u[EPI_RUN];
#pragma unroll
    for (int j = 0; j < EPI_RUN; ++j) {
        const int64_t n = n0 + j < N ? n0 + j : N - 1;
        col[j] = column(e, n);
#pragma unroll
        for (int k = 0; k < 4; ++k) yz[j][k] = *(const v4f *)(col[j].nb[2 + k] + q);
        u[j] = *(const v4f *)(U + n * Q + q);
    }
#pragma unroll
    for (int j = 0; j < EPI_RUN; ++j) {
        if (n0 + j >= N) break;
        // a missing x-neighbour is the voxel's own row at weight 0, as in column()
        const v4f nb[6] = {col[j].wt[0] != 0.0f ? xr[j] : xr[j + 1], col[j].wt[1] != 0.0f ? xr[j + 2] : xr[j + 1],
                           yz[j][0], yz[j][1], yz[j][2], yz[j][3]};
        zupdate(e, col[j], q, xr[j + 1], nb, u[j]);
    }
}

__global__ void __launch_bounds__(256)
k_epi_w(EpiW e, const float *__restrict__ Y, int64_t N) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int per = e.Rg / 4;
    if (idx >= N * per) return;
    const int64_t n = idx / per;
    const int q[1] = {4 * (int)(idx % per)};
    const v4f y[1] = {*(const v4f *)(Y + n * (int64_t)e.Rg + q[0])};
    epilogue_batch<1>(e, column(e, n), q, y);
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

// f and d around iteration k of the library path (voxel-major rows of Qg, the
// product's u^k = V_r w^k still in its buffer): t = z^k + u^k, f^{k+1} = t -
// d^k / beta (written over d^k in place when f is given; d^0 = 0 when dprev is
// NULL) and d^{k+1} = beta (t - z^{k+1}) (Algorithm 2's f- and d-steps in the
// reduced form).
__global__ void __launch_bounds__(256)
k_gemm_aux(const float *z, const float *u, const float *zn, const float *dprev, float *f, float *d,
           size_t count, float beta) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float t = z[i] + u[i];
    if (f) f[i] = t - (dprev ? dprev[i] : 0.0f) / beta;
    d[i] = beta * (t - zn[i]);
}

}  // namespace

namespace {

// M x K by N x K product with epilogue e; false for shapes the tiles do not cover.
template <typename E>
bool gemm_tn(bool bf16, const void *A, const void *B, int M, int K, int KB, int64_t N, const E &e,
             hipStream_t s) {
    const int KT = bf16 ? GK<uint16_t>::KT : GK<float>::KT;
    if (M % 128 || K % KT || KB % KT || KB <= 0 || KB > K || N <= 0) return false;
    if ((N + 127) / 128 * (M / 128) > 0x7fffffff) return false;   // one-dimensional grid
    const dim3 block(GNT);
    const unsigned nb = nblocks(N, 128);
    if (bf16 && M % 256 == 0) {
        // 256 x 128 workgroup tiles, 128 x 64 per wave
        hipLaunchKernelGGL((k_gemm_tn<uint16_t, 8, 4, E>), dim3(nb * (unsigned)(M / 256)), block, 0, s,
                           (const uint16_t *)A, (const uint16_t *)B, M, K, KB, N, e);
    } else if (bf16) {
        hipLaunchKernelGGL((k_gemm_tn<uint16_t, 4, 4, E>), dim3(nb * (unsigned)(M / 128)), block, 0, s,
                           (const uint16_t *)A, (const uint16_t *)B, M, K, KB, N, e);
    } else {
        hipLaunchKernelGGL((k_gemm_tn<float, 4, 4, E>), dim3(nb * (unsigned)(M / 128)), block, 0, s,
                           (const float *)A, (const float *)B, M, K, KB, N, e);
    }
    return true;
}

}  // namespace

bool launch_gemm_u(bool bf16, const void *A, const void *B, int K, const float *z, float *zn,
                   uint16_t *zs, Grid g, int Qg, double tau, double lam2, double beta,
                   const uint8_t *code, hipStream_t s) {
    const EpiZ e{z, zn, zs, g, Qg, (float)tau, (float)lam2, (float)beta, code, 2};
    return gemm_tn(bf16, A, B, Qg, K, bf16 ? K / 3 * 2 : K, g.N, e, s);
}

bool launch_gemm_y(bool bf16, const void *A, const void *B, int K, int64_t N, int Rg, const float *ah,
                   float *sv, float *w, uint16_t *ws, const float *bcoef, hipStream_t s) {
    const EpiW e{ah, sv, w, ws, bcoef, Rg, 2};
    return gemm_tn(bf16, A, B, Rg, K, bf16 ? K / 3 * 2 : K, N, e, s);
}

void launch_epi_z(const float *U, const float *z, float *zn, uint16_t *zs3, Grid g, int Qg, double tau,
                  double lam2, double beta, const uint8_t *code, hipStream_t s) {
    const EpiZ e{z, zn, zs3, g, Qg, (float)tau, (float)lam2, (float)beta, code, 3};
    const int64_t qt = (Qg / 4 + 255) / 256;
    hipLaunchKernelGGL(k_epi_z, dim3((unsigned)(nblocks(g.N, EPI_RUN) * qt)), dim3(256), 0, s, e, U);
}

void launch_epi_w(const float *Y, int64_t N, int Rg, const float *ah, float *sv, float *w, uint16_t *ws3,
                  const float *bcoef, hipStream_t s) {
    const EpiW e{ah, sv, w, ws3, bcoef, Rg, 3};
    hipLaunchKernelGGL(k_epi_w, dim3(nblocks(N * (Rg / 4), 256)), dim3(256), 0, s, e, Y, N);
}

void launch_gemm_aux(const float *z, const float *u, const float *zn, const float *dprev, float *f,
                     float *d, size_t count, double beta, hipStream_t s) {
    hipLaunchKernelGGL(k_gemm_aux, dim3(nblocks((int64_t)count, 256)), dim3(256), 0, s, z, u, zn, dprev, f,
                       d, count, (float)beta);
}

void launch_gemm_from_ranks(const float *src, int RP, float *dst, uint16_t *ds, int64_t N, int Rg,
                            hipStream_t s, int nseg) {
    hipLaunchKernelGGL(k_gemm_from_ranks, dim3(nblocks(N * Rg, 256)), dim3(256), 0, s, src, RP, dst, ds,
                       N, Rg, nseg);
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
