// Setup, monitoring and output kernels shared by both iteration kernels,
// and the unfused reference iteration (two passes per iteration, any rank).
//
// The iteration is Algorithm 2 (Sec. III-E) written in a reduced form that
// gives the same iterates in exact arithmetic. With K_r = U_r S_r V_r^T,
// h_n = S_r U_r^T m_n (so g_n = V_r h_n), a_i = 1/(beta + s_i^2) and
// b_i = s_i^2/(beta + s_i^2) (the two parts of the weights of
// Eq. DictVecSVD), the f-step becomes
//     f^{k+1} = z^k - d^k/beta + V_r w^k,  w^k = a.h - b.(V_r^T z^k - V_r^T d^k/beta).
// Substituting f into the z-step of Eq. (z2) cancels d exactly:
//     z^{k+1} = max(0, z^k - tau (lambda D^T D z^k - beta V_r w^k)),  tau = 1/(xi_p + beta),
//     d^{k+1} = beta (z^k - z^{k+1} + V_r w^k),
// and, with y^k = V_r^T z^k, the r-vector recursion
//     w^{k+1} = a.h - b.(2 y^{k+1} - y^k - w^k),  w^0 = a.h,  y^0 = 0.
// Only z (Q per voxel) and three r-vectors per voxel are kept, and the form
// has no c/beta - V(s.V^T c) cancellation, so it holds accuracy in float32.
#include "internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

namespace ssmap {

namespace {

template <int MODE> struct StateT { using T = float; };
template <> struct StateT<MODE_FP64> { using T = double; };

// bf16 round-to-nearest-even of a float, returned as a float (low 16 bits 0).
__device__ __forceinline__ float bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

// Product used by the contractions. MODE_BF16X3 emulates the three-term
// split product hi*hi + hi*lo + lo*hi that the MFMA path evaluates.
template <int MODE, typename T>
__device__ __forceinline__ T cprod(T v, T x) {
    if constexpr (MODE == MODE_BF16X3) {
        const float vh = bf16_rne(v), vl = bf16_rne(v - vh);
        const float xh = bf16_rne(x), xl = bf16_rne(x - xh);
        return vh * xh + (vh * xl + vl * xh);
    } else {
        return v * x;
    }
}

__device__ __forceinline__ int64_t chunk_index(int q, int64_t n, int64_t N) {
    return ((int64_t)(q / QC) * N + n) * QC + (q % QC);
}

// ------------------------------------------------------------- projection
// t_n = U_r^T m_n (float64 accumulation in increasing p), ah = w = a .* (s .* t),
// y = 0, optional t and ||m_n||^2 - ||t_n||^2, and the non-finite flag.
// A block takes 64 voxels and 4 rank groups of 8 ranks (32 ranks per pass over
// M; ranks above 32 take further passes). M arrives voxel-major (row n holds
// P measurements), so tiles of 64 voxels x 32 measurements are read as
// 128-byte row segments and stored transposed in LDS, where a wave reads one
// measurement of its 64 voxels without bank conflicts; the matching rows of
// U_r are broadcast from LDS.
constexpr int PJ_V = 64, PJ_P = 32, PJ_G = 4, PJ_R = 8;

template <int MODE>
__global__ void __launch_bounds__(256)
k_project(const typename StateT<MODE>::T *__restrict__ M, int P,
          const double *__restrict__ Ur, const double *__restrict__ sig,
          const double *__restrict__ acoef, int r, int RP, int64_t N,
          double *__restrict__ t, double *__restrict__ mperp2,
          typename StateT<MODE>::T *__restrict__ ah, typename StateT<MODE>::T *__restrict__ w,
          typename StateT<MODE>::T *__restrict__ y, int *__restrict__ bad,
          const uint8_t *__restrict__ code) {
    using T = typename StateT<MODE>::T;
    constexpr int RW = PJ_G * PJ_R;                     // ranks per pass
    __shared__ double Ms[PJ_P][PJ_V + 1];
    __shared__ double Us[PJ_P][RW];
    __shared__ double red[PJ_G][PJ_V];
    const int tid = threadIdx.x, v = tid & (PJ_V - 1), g = tid / PJ_V;
    const int64_t n0 = (int64_t)blockIdx.x * PJ_V, n = n0 + v;
    // outside voxels of a mask are not estimated: zeros, data not read
    auto inside = [&](int64_t k) { return k < N && (!code || (code[k] & 0x80u) != 0); };
    double msq = 0.0, tsq = 0.0;
    bool finite = true;
    for (int i0 = 0; i0 < r; i0 += RW) {
        double acc[PJ_R];
#pragma unroll
        for (int j = 0; j < PJ_R; ++j) acc[j] = 0.0;
        for (int p0 = 0; p0 < P; p0 += PJ_P) {
            __syncthreads();                                // the previous tile is consumed
#pragma unroll
            for (int k = 0; k < PJ_V * PJ_P / 256; ++k) {
                const int e = tid + 256 * k, row = e / PJ_P, col = e % PJ_P;
                const int64_t nn = n0 + row;
                const int pp = p0 + col;
                Ms[col][row] = (inside(nn) && pp < P) ? (double)M[nn * P + pp] : 0.0;
            }
            for (int e = tid; e < PJ_P * RW; e += 256) {
                const int pp = p0 + e / RW, ii = i0 + e % RW;
                Us[e / RW][e % RW] = (pp < P && ii < r) ? Ur[(size_t)pp * r + ii] : 0.0;
            }
            __syncthreads();
            const int pend = min(PJ_P, P - p0);
            if (i0 == 0 && g == 0)
                for (int p = 0; p < pend; ++p) {
                    const double x = Ms[p][v];
                    finite &= __builtin_isfinite(x);
                    msq += x * x;
                }
            for (int p = 0; p < pend; ++p) {
                const double x = Ms[p][v];
#pragma unroll
                for (int j = 0; j < PJ_R; ++j) acc[j] += Us[p][g * PJ_R + j] * x;
            }
        }
#pragma unroll
        for (int j = 0; j < PJ_R; ++j) {
            const int i = i0 + g * PJ_R + j;
            if (n < N && i < r) {        // outside voxels accumulated zeros
                tsq += acc[j] * acc[j];
                if (t) t[(size_t)i * N + n] = acc[j];
                const T val = (T)(acoef[i] * (sig[i] * acc[j]));
                ah[(size_t)i * N + n] = val;
                w[(size_t)i * N + n] = val;
                y[(size_t)i * N + n] = (T)0;
            }
        }
    }
    if (n < N)
        for (int i = r + g; i < RP; i += PJ_G) {
            ah[(size_t)i * N + n] = (T)0;
            w[(size_t)i * N + n] = (T)0;
            y[(size_t)i * N + n] = (T)0;
        }
    if (!finite) atomicOr(bad, 1);
    if (mperp2) {                                       // uniform over the block
        red[g][v] = tsq;
        __syncthreads();
        if (g == 0 && n < N) mperp2[n] = msq - (((red[0][v] + red[1][v]) + red[2][v]) + red[3][v]);
    }
}

// ------------------------------------------------------------- unfused iteration
// Pass 1: for each (q, n): u = (V_r w)_q, the D^T D stencil on plane q,
// the projected z-update, and optionally d^{k+1} and f^{k+1}.
template <int MODE>
__global__ void __launch_bounds__(256)
k_update(IterArgs a) {
    using T = typename StateT<MODE>::T;
    const int64_t N = a.g.N;
    const int c = blockIdx.y;
    const int64_t local = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (local >= N * QC) return;
    const int64_t n = local / QC;
    const int qq = (int)(local % QC);
    const int q = c * QC + qq;
    const int64_t e = ((int64_t)c * N + n) * QC + qq;
    const T *z = (const T *)a.z;
    const T *V = (const T *)a.V + (size_t)q * a.RP;
    const T *w = (const T *)a.w;
    T u = 0;
    for (int i = 0; i < a.r; ++i) u += cprod<MODE>(V[i], w[(size_t)i * N + n]);
    const T zc = z[e];
    const int64_t nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const int64_t x = n % nx, yy = (n / nx) % ny, zz = n / (nx * ny);
    T lap = 0;
    bool inside = true;
    if (a.code) {
        // masked grid: outside voxels hold z = 0, so summing every box
        // neighbour and taking the inside-neighbour count is exact
        const unsigned cb = a.code[n];
        inside = (cb & 0x80u) != 0;
        T nsum = 0;
        if (x > 0) nsum += z[e - QC];
        if (x < nx - 1) nsum += z[e + QC];
        if (yy > 0) nsum += z[e - nx * QC];
        if (yy < ny - 1) nsum += z[e + nx * QC];
        if (zz > 0) nsum += z[e - nx * ny * QC];
        if (zz < nz - 1) nsum += z[e + nx * ny * QC];
        lap = (T)(cb & 7u) * zc - nsum;
    } else {
        if (x > 0) lap += zc - z[e - QC];
        if (x < nx - 1) lap += zc - z[e + QC];
        if (yy > 0) lap += zc - z[e - nx * QC];
        if (yy < ny - 1) lap += zc - z[e + nx * QC];
        if (zz > 0) lap += zc - z[e - nx * ny * QC];
        if (zz < nz - 1) lap += zc - z[e + nx * ny * QC];
    }
    const T tau = (T)a.tau, lam2 = (T)a.lam2, beta = (T)a.beta;
    T zn = zc - tau * (lam2 * lap - beta * u);
    zn = (zn > (T)0 && inside) ? zn : (T)0;
    ((T *)a.znew)[e] = zn;
    if (a.fout) {
        const T dp = a.dprev ? ((const T *)a.dprev)[e] : (T)0;
        ((T *)a.fout)[e] = zc + u - dp / beta;
    }
    if (a.dout) ((T *)a.dout)[e] = beta * (zc - zn + u);
}

// Pass 2: y^{k+1} = V_r^T z^{k+1} per voxel and the w recursion.
template <int MODE, int RB>
__global__ void __launch_bounds__(256)
k_projw(IterArgs a) {
    using T = typename StateT<MODE>::T;
    const int64_t N = a.g.N;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const T *zn = (const T *)a.znew;
    const T *V = (const T *)a.V;
    const T *b = (const T *)a.bcoef;
    const T *ah = (const T *)a.ah;
    T *w = (T *)a.w;
    T *y = (T *)a.y;
    for (int i0 = 0; i0 < a.r; i0 += RB) {
        T acc[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) acc[j] = 0;
        for (int c = 0; c < a.nchunk; ++c) {
            const T *zp = zn + ((int64_t)c * N + n) * QC;
            for (int qq = 0; qq < QC; ++qq) {
                const T zv = zp[qq];
                const T *vrow = V + (size_t)(c * QC + qq) * a.RP + i0;
#pragma unroll
                for (int j = 0; j < RB; ++j)
                    if (i0 + j < a.RP) acc[j] += cprod<MODE>(vrow[j], zv);
            }
        }
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            const int i = i0 + j;
            if (i < a.r) {
                const size_t o = (size_t)i * N + n;
                const T yn = acc[j];
                w[o] = ah[o] - b[i] * ((T)2 * yn - y[o] - w[o]);
                y[o] = yn;
            }
        }
    }
}

// ------------------------------------------------------------- aux (f, d) around a fused pass
// The fused iteration never materialises f or d. When f^K and d^K are asked
// for, the last two iterations are bracketed by these passes:
//   before iteration k:  t = z^k + V_r w^k            (and f^{k+1} = t - d^k / beta)
//   after  iteration k:  d^{k+1} = beta (t - z^{k+1})
template <int MODE>
__global__ void __launch_bounds__(256)
k_aux_pre(IterArgs a, typename StateT<MODE>::T *__restrict__ t, typename StateT<MODE>::T *f,
          const typename StateT<MODE>::T *dprev) {
    using T = typename StateT<MODE>::T;
    const int64_t N = a.g.N;
    const int c = blockIdx.y;
    const int64_t local = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (local >= N * QC) return;
    const int64_t n = local / QC;
    const int q = c * QC + (int)(local % QC);
    const int64_t e = ((int64_t)c * N + n) * QC + (local % QC);
    const T *V = (const T *)a.V + (size_t)q * a.RP;
    const T *w = (const T *)a.w;
    T u = 0;
    for (int i = 0; i < a.r; ++i) u += cprod<MODE>(V[i], w[(size_t)i * N + n]);
    const T tv = ((const T *)a.z)[e] + u;
    t[e] = tv;
    if (f) {
        const T dp = dprev ? dprev[e] : (T)0;
        f[e] = tv - dp / (T)a.beta;
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_aux_post(T *__restrict__ t, const T *__restrict__ znew, T beta, size_t count) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) t[i] = beta * (t[i] - znew[i]);
}

// ------------------------------------------------------------- monitoring
// Objective of Eq. (spat) with R of Eq. (l2), residuals and DFCS (Eq. DFCS) of
// an iterate, all summed in float64. A wave takes 16 consecutive voxels at a
// time; lane l holds voxel l % 16 and the four nodes 4 (l / 16) .. + 3 of each
// 16-node chunk. The data term uses
//     ||m_n - K_r z_n||^2 = ||m_n||^2 - ||t_n||^2 + sum_i (t_i - sigma_i y_i)^2,
// t = U_r^T m_n, y = V_r^T z_n. The iteration kernels leave y of the new iterate
// in their r-vector state (contracted there in the state precision; the objective
// then differs from the float64 contraction by about 1e-8 relative in float32
// and 1e-6 in bf16x3), which the monitor reads when it is given. Otherwise (the
// GEMM path keeps no y) y is contracted here on the matrix cores in float64
// (v_mfma_f64_16x16x4: M = 16 ranks, N = 16 voxels, K = 4 nodes; the lane's own
// z values are the B operand, K-row l / 16 of step s being node 4 (l / 16) + s;
// output rank 16 rb + l / 16 + 4 i in lane l). The regulariser
// takes every forward face edge once (both ends inside a mask). Sums are
// reduced across the wave by shuffles, across the four waves through LDS,
// then in a fixed order over the blocks, so every result is bitwise repeatable.
// SP (small grids with y given): a block takes one 16-voxel tile and its four
// waves split the chunks (c = wave mod 4) and the ranks (r = lane / 16 + 4 wave
// mod 16), a quarter of the serial loads per wave where the few tiles would
// leave most CUs idle.
typedef double v4d_m __attribute__((ext_vector_type(4)));

template <typename T, bool VM>
__device__ __forceinline__ void load4(const T *base, int64_t off, bool ok, T out[4]) {
    if constexpr (sizeof(T) == 4) {
        const float4 v = ok ? *(const float4 *)(base + off) : float4{0.f, 0.f, 0.f, 0.f};
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else {
        const double2 a = ok ? *(const double2 *)(base + off) : double2{0.0, 0.0};
        const double2 b = ok ? *(const double2 *)(base + off + 2) : double2{0.0, 0.0};
        out[0] = a.x; out[1] = a.y; out[2] = b.x; out[3] = b.y;
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

constexpr int MON_RG = 4;                // 16-rank blocks per pass over z

// 16 bytes (four float or two double values) through a raw buffer resource;
// offsets are 32-bit within one chunk of the state
__device__ __forceinline__ __amdgpu_buffer_rsrc_t mon_rsrc(const void *p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ void bload4(__amdgpu_buffer_rsrc_t r, unsigned off, T out[4]) {
    typedef unsigned v4u_m __attribute__((ext_vector_type(4)));
    const v4u_m a = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) out[i] = __uint_as_float(a[i]);
    } else {
        const v4u_m b = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, 0);
        out[0] = __hiloint2double(a[1], a[0]);
        out[1] = __hiloint2double(a[3], a[2]);
        out[2] = __hiloint2double(b[1], b[0]);
        out[3] = __hiloint2double(b[3], b[2]);
    }
}
constexpr unsigned MON_OOB = 0x80000000u;   // beyond every range: loads return 0

template <typename T, bool VM, bool SP>
__global__ void __launch_bounds__(256)
k_monitor(MonArgs a, double *__restrict__ partial) {
    const T *z = (const T *)a.z;
    const T *zp = (const T *)a.zprev;
    const T *fz = (const T *)a.f;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = lane & 15, i4 = lane >> 4;
    const int64_t N = a.g.N, nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const int RB = a.RP / 16;
    // element (q, n): chunked z[((q / 16) N + n) 16 + q % 16], or voxel-major z[n ld + q]
    auto at = [&](int c, int64_t n) -> int64_t {
        return VM ? n * a.ld + 16 * c + 4 * i4 : ((int64_t)c * N + n) * QC + 4 * i4;
    };
    auto in = [&](int64_t v) { return !a.code || (a.code[v] & 0x80u) != 0; };
    double acc[ST_COUNT];
#pragma unroll
    for (int k = 0; k < ST_COUNT; ++k) acc[k] = 0.0;
    const int64_t ntile = (N + 15) / 16;
    const int64_t t0 = SP ? (int64_t)blockIdx.x : (int64_t)blockIdx.x * 4 + wave;
    const int64_t tstep = SP ? (int64_t)gridDim.x : (int64_t)gridDim.x * 4;
    const int c0 = SP ? wave : 0, cstep = SP ? 4 : 1;             // chunks of this wave
    const int r0 = SP ? i4 + 4 * wave : i4, rstep = SP ? 16 : 4;  // ranks of this wave
    for (int64_t tile = t0; tile < ntile; tile += tstep) {
        const int64_t n = tile * 16 + j;
        const bool valid = n < N;
        const int64_t x = n % nx, yy = (n / nx) % ny, zz = n / (nx * ny);
        const bool ein = valid && in(n);
        const bool ex = ein && x + 1 < nx && in(n + 1);
        const bool ey = ein && yy + 1 < ny && in(n + nx);
        const bool ez = ein && zz + 1 < nz && in(n + nx * ny);
        const bool contract = a.y == nullptr && a.ypart == nullptr;
        if (!contract && valid)             // data term from the iteration's y
            for (int rr = r0; rr < a.r; rr += rstep) {
                const double tv = a.t[(size_t)rr * N + n], sg = a.sig[rr];   // with the y loads
                double yv;
                if (SP && a.ypart) {        // the same sums, every load unconditional (out of range: 0)
                    T ys = (T)0;
                    const __amdgpu_buffer_rsrc_t pr =
                        mon_rsrc(a.ypart, (unsigned)((size_t)a.npart * a.RP * N * sizeof(T)));
                    for (int c0 = 0; c0 < a.npart; c0 += 8) {
                        T pv[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const unsigned off = ein && c0 + u < a.npart
                                ? (unsigned)((((size_t)(c0 + u) * a.RP + rr) * N + n) * sizeof(T)) : MON_OOB;
                            if constexpr (sizeof(T) == 8)
                                pv[u] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(pr, off, 0, 0));
                            else
                                pv[u] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(pr, off, 0, 0));
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u) ys += pv[u];
                    }
                    yv = (double)ys;
                } else if (a.ypart) {       // the partials in chunk order, as the next iteration sums them
                    T ys = (T)0;            // (bricks outside a mask are never written; z = y = 0 there)
                    const T *yp = (const T *)a.ypart + (size_t)rr * N + n;
                    for (int c0 = 0; ein && c0 < a.npart; c0 += 8) {
                        T pv[8];            // eight loads in flight, then added in order
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            pv[u] = c0 + u < a.npart ? yp[(size_t)(c0 + u) * a.RP * N] : (T)0;
#pragma unroll
                        for (int u = 0; u < 8; ++u) ys += pv[u];
                    }
                    yv = (double)ys;
                } else {
                    yv = (double)((const T *)a.y)[a.yld > 0 ? (size_t)n * a.yld + rr : (size_t)rr * N + n];
                }
                const double e = tv - sg * yv;
                acc[ST_DATA] += e * e;
            }
        // this lane's sums over its four nodes of chunk c: z norm, non-finite count,
        // regulariser, dual, primal and DFCS terms
        auto mon_stats = [&](int c, const T (&zv)[4], const T (&nb)[3][4], const T (&pv)[4],
                             const T (&fv)[4]) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const double v = (double)zv[s];
                if (!__builtin_isfinite(v)) acc[ST_NONFINITE] += 1.0;
                acc[ST_ZNORM] += v * v;
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    const double dd = v - (double)nb[e][s];
                    acc[ST_REG] += (e == 0 ? ex : e == 1 ? ey : ez) ? dd * dd : 0.0;
                }
                if (zp) {
                    const double dd = v - (double)pv[s];
                    acc[ST_DZ] += dd * dd;
                }
                const int q = 16 * c + 4 * i4 + s;
                const bool has_ref = a.fstar && valid && q < a.Q;
                const double fs = has_ref ? a.fstar[n * a.Q + q] : 0.0;
                if (a.fstar) {
                    const double dd = has_ref ? v - fs : 0.0;
                    acc[ST_DFCS] += dd * dd;
                    acc[ST_FSTAR] += fs * fs;
                }
                if (fz) {
                    const double f = (double)fv[s];
                    const double dd = v - f;
                    acc[ST_PRIMAL] += dd * dd;
                    if (a.fstar) {
                        const double df = has_ref ? f - fs : 0.0;
                        acc[ST_DFCS_F] += df * df;
                    }
                }
            }
        };
        for (int rg = 0; rg < RB || rg == 0; rg += MON_RG) {
            if (!contract && rg > 0) break;
            v4d_m yacc[MON_RG];
#pragma unroll
            for (int g = 0; g < MON_RG; ++g) yacc[g] = v4d_m{0.0, 0.0, 0.0, 0.0};
            for (int c = c0; c < a.nchunk; c += cstep) {
                T zv[4];
                if constexpr (SP) {
                    // every load of the step issues before any is used (out of range: 0);
                    // the host keeps these arrays below 2^31 bytes
                    const unsigned zb = (unsigned)((VM ? N * a.ld : (int64_t)a.nchunk * N * QC) * sizeof(T));
                    const __amdgpu_buffer_rsrc_t zr = mon_rsrc(z, zb), pr = mon_rsrc(zp ? zp : z, zb),
                                                 fr = mon_rsrc(fz ? fz : z, zb);
                    auto bo = [&](int64_t e, bool ok) { return ok ? (unsigned)(e * sizeof(T)) : MON_OOB; };
                    T nb[3][4], pv[4], fv[4];
                    bload4<T>(zr, bo(at(c, n), valid), zv);
                    bload4<T>(zr, bo(at(c, n + 1), ex), nb[0]);
                    bload4<T>(zr, bo(at(c, n + nx), ey), nb[1]);
                    bload4<T>(zr, bo(at(c, n + nx * ny), ez), nb[2]);
                    bload4<T>(pr, bo(at(c, n), valid && zp), pv);
                    bload4<T>(fr, bo(at(c, n), valid && fz), fv);
                    mon_stats(c, zv, nb, pv, fv);
                    continue;                   // no contraction here: y is given
                }
                load4<T, VM>(z, at(c, n), valid, zv);
                if (rg == 0) {
                    T nb[3][4], pv[4], fv[4];
                    load4<T, VM>(z, at(c, n + 1), ex, nb[0]);
                    load4<T, VM>(z, at(c, n + nx), ey, nb[1]);
                    load4<T, VM>(z, at(c, n + nx * ny), ez, nb[2]);
                    if (zp) load4<T, VM>(zp, at(c, n), valid, pv);
                    if (fz) load4<T, VM>(fz, at(c, n), valid, fv);
                    mon_stats(c, zv, nb, pv, fv);
                }
                // y of ranks 16 (rg + g) .. + 15 over this chunk's 16 nodes
#pragma unroll
                for (int g = 0; g < MON_RG; ++g) {
                    const int rb = rg + g;
                    if (contract && rb < RB) {
                        const double *Vc = a.V64 + (size_t)(16 * c + 4 * i4) * a.RP + 16 * rb + j;
#pragma unroll
                        for (int s = 0; s < 4; ++s)
                            yacc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(Vc[(size_t)s * a.RP],
                                                                          (double)zv[s], yacc[g], 0, 0, 0);
                    }
                }
            }
#pragma unroll
            for (int g = 0; g < MON_RG; ++g)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int rr = 16 * (rg + g) + i4 + 4 * i;
                    if (contract && valid && rr < a.r) {
                        const double e = a.t[(size_t)rr * N + n] - a.sig[rr] * yacc[g][i];
                        acc[ST_DATA] += e * e;
                    }
                }
        }
        if (valid && i4 == 0 && (!SP || wave == 0)) acc[ST_DATA] += a.mperp2[n];
    }
    __shared__ double red[4][ST_COUNT];
#pragma unroll
    for (int k = 0; k < ST_COUNT; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < ST_COUNT) {
        const int k = threadIdx.x;
        partial[(size_t)blockIdx.x * ST_COUNT + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

// The same sums for the chunked layout when the iteration left y, in one pass
// that reads each value of z about once. A column is one 16 x 16 voxel tile of
// one chunk over all z-planes; a block marches a column along z. Each lane holds
// one quarter (four values) of a voxel's 16-node chunk row in four rows of the
// tile (rows 4 wave .. 4 wave + 3). The x neighbour comes from the lane four
// places on (the tile's last column reads the next tile's first voxel), the y
// neighbour from the lane's next row (its last row reads the row after it, which
// the next wave also loads), and the z neighbour is the next plane, which the
// block loads for this plane and keeps for the next. Workgroups are dealt to the
// eight XCDs in turn (block b on XCD b mod 8): each XCD takes a contiguous run of
// columns and its blocks march neighbouring columns side by side, so the halo
// rows one block reads are those its neighbours load at about the same time,
// through the XCD's L2. Squares are summed in the state precision over a plane,
// then accumulated in float64; the per-voxel data term from y and t is spread
// over all blocks. EXTRA: zprev, f or the reference map may be given (the build
// without them holds fewer registers and runs more waves).
constexpr int MT_X = 16, MT_Y = 16, MT_RW = 4;
template <typename T, bool EXTRA>
__global__ void __launch_bounds__(256)
k_monitor_march(MonArgs a, double *__restrict__ partial) {
    const uint32_t N = (uint32_t)a.g.N, nx = (uint32_t)a.g.nx, ny = (uint32_t)a.g.ny,
                   nz = (uint32_t)a.g.nz, nxy = nx * ny;
    const unsigned cbytes = (unsigned)((size_t)N * QC * sizeof(T));
    constexpr unsigned kFar = 0x80000000u;   // beyond every chunk: the buffer load returns 0
    const bool hasp = EXTRA && a.zprev != nullptr, hasf = EXTRA && a.f != nullptr,
               hasr = EXTRA && a.fstar != nullptr;
    auto in = [&](uint32_t v) { return !a.code || (a.code[v] & 0x80u) != 0; };
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t qd = lane & 3, xv = lane >> 2;
    double acc[ST_COUNT];
#pragma unroll
    for (int k = 0; k < ST_COUNT; ++k) acc[k] = 0.0;
    const uint32_t ntx = (nx + MT_X - 1) / MT_X, nty = (ny + MT_Y - 1) / MT_Y, ntile = ntx * nty;
    // columns of this block: XCD x = b mod 8 owns [x cx, (x + 1) cx); its gx blocks take
    // columns l, l + gx, ... of that run (gridDim.x = 8 gx)
    const uint32_t ncol = ntile * (uint32_t)a.nchunk, cx = (ncol + 7) / 8, gx = gridDim.x / 8;
    const uint32_t xcd = blockIdx.x & 7, col_end = min(ncol, (xcd + 1) * cx);
    const unsigned sx = QC * sizeof(T), sz = nxy * QC * sizeof(T);
    T cur[MT_RW][4];
    bool have = false;
    uint32_t col = xcd * cx + (blockIdx.x >> 3), zz = 0;
    for (; col < col_end; zz = zz + 1 < nz ? zz + 1 : 0, col += zz == 0 ? gx : 0) {
        const uint32_t c = col / ntile, tile = col - c * ntile;
        const uint32_t x = (tile % ntx) * MT_X + xv, y0 = (tile / ntx) * MT_Y + MT_RW * wave;
        const size_t cbase = (size_t)c * N * QC;
        const __amdgpu_buffer_rsrc_t zr = mon_rsrc((const T *)a.z + cbase, cbytes);
        const bool xok = x < nx, znext = zz + 1 < nz;
        // byte offset of this lane's quarter at row y0 + j of plane zz (kFar outside the grid)
        unsigned off[MT_RW];
#pragma unroll
        for (int j = 0; j < MT_RW; ++j)
            off[j] = (xok && y0 + j < ny) ? ((x + nx * (y0 + j + ny * zz)) * QC + 4 * qd) * (unsigned)sizeof(T)
                                          : kFar;
        if (!have)
#pragma unroll
            for (int j = 0; j < MT_RW; ++j) bload4<T>(zr, off[j], cur[j]);
        // the next plane (z neighbours), the row after the lane's last (y neighbours) and,
        // in the tile's last column, the voxel after it (x neighbours)
        T nxt[MT_RW][4], yx[4], hx[MT_RW][4];
#pragma unroll
        for (int j = 0; j < MT_RW; ++j) bload4<T>(zr, znext && off[j] != kFar ? off[j] + sz : kFar, nxt[j]);
        bload4<T>(zr, (xok && y0 + MT_RW < ny) ? ((x + nx * (y0 + MT_RW + ny * zz)) * QC + 4 * qd) *
                                                     (unsigned)sizeof(T)
                                               : kFar, yx);
        const bool halo = xv == MT_X - 1 && x + 1 < nx;
#pragma unroll
        for (int j = 0; j < MT_RW; ++j) {
            if (halo) bload4<T>(zr, off[j] != kFar ? off[j] + sx : kFar, hx[j]);
            else
#pragma unroll
                for (int s = 0; s < 4; ++s) hx[j][s] = 0;
        }
        T zsq = 0, reg = 0, dsq = 0, psq = 0;
#pragma unroll
        for (int j = 0; j < MT_RW; ++j) {
            const uint32_t yj = y0 + j, n = x + nx * (yj + ny * zz);
            const bool ein = off[j] != kFar && in(n);
            const bool ex = ein && x + 1 < nx && in(n + 1);
            const bool ey = ein && yj + 1 < ny && in(n + nx);
            const bool ez = ein && znext && in(n + nxy);
            T pv[4], fv[4];
            if (hasp) bload4<T>(mon_rsrc((const T *)a.zprev + cbase, cbytes), off[j], pv);
            if (hasf) bload4<T>(mon_rsrc((const T *)a.f + cbase, cbytes), off[j], fv);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const T v = cur[j][s];
                const T sh = __shfl_down(v, 4, 64);          // same quarter, voxel x + 1
                const T xn = halo ? hx[j][s] : sh;
                const T yn = j + 1 < MT_RW ? cur[j + 1 < MT_RW ? j + 1 : j][s] : yx[s];
                zsq += v * v;
                const T d0 = ex ? v - xn : (T)0, d1 = ey ? v - yn : (T)0, d2 = ez ? v - nxt[j][s] : (T)0;
                reg += d0 * d0 + d1 * d1 + d2 * d2;
                if (hasp) {
                    const T dd = v - pv[s];
                    dsq += dd * dd;
                }
                if (hasf) {
                    const T dd = v - fv[s];
                    psq += dd * dd;
                }
            }
            if (hasr && off[j] != kFar) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int q = 16 * (int)c + 4 * (int)qd + s;
                    const double fs = q < a.Q ? a.fstar[(size_t)n * a.Q + q] : 0.0;
                    const double dd = q < a.Q ? (double)cur[j][s] - fs : 0.0;
                    acc[ST_DFCS] += dd * dd;
                    acc[ST_FSTAR] += fs * fs;
                    if (hasf) {
                        const double df = q < a.Q ? (double)fv[s] - fs : 0.0;
                        acc[ST_DFCS_F] += df * df;
                    }
                }
            }
        }
        // a NaN or Inf anywhere in the unit (or a square beyond the state type's range)
        // leaves the unit's sum of squares non-finite
        acc[ST_NONFINITE] += __builtin_isfinite(zsq) ? 0.0 : 1.0;
        acc[ST_ZNORM] += (double)zsq;
        acc[ST_REG] += (double)reg;
        acc[ST_DZ] += (double)dsq;
        acc[ST_PRIMAL] += (double)psq;
#pragma unroll
        for (int j = 0; j < MT_RW; ++j)
#pragma unroll
            for (int s = 0; s < 4; ++s) cur[j][s] = nxt[j][s];
        have = znext;
    }
    {                                        // data term: ||m_perp||^2 + sum_i (t_i - sigma_i y_i)^2,
        const T *y = (const T *)a.y;         // voxels spread over every block of the grid
        const uint32_t all = gridDim.x * blockDim.x;
        for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += all) {
            double d = a.mperp2[n];
            for (int i = 0; i < a.r; ++i) {
                const double e = a.t[(size_t)i * N + n] - a.sig[i] * (double)y[(size_t)i * N + n];
                d += e * e;
            }
            acc[ST_DATA] += d;
        }
    }
    __shared__ double red[4][ST_COUNT];
#pragma unroll
    for (int k = 0; k < ST_COUNT; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < ST_COUNT) {
        const int k = threadIdx.x;
        partial[(size_t)blockIdx.x * ST_COUNT + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

// Fixed-order sum of the per-block partials: thread t adds blocks t, t + 256, ...
// in turn; then shuffles within each wave and the four wave sums in order.
__global__ void __launch_bounds__(256)
k_reduce_partials(const double *__restrict__ partial, int nblocks, const double *__restrict__ dzpart,
                  int ndz, double *__restrict__ out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ double red[4][ST_COUNT];
    double acc[ST_COUNT];
#pragma unroll
    for (int k = 0; k < ST_COUNT; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < ST_COUNT; ++k) acc[k] += partial[(size_t)b * ST_COUNT + k];
    if (dzpart)                              // the iteration's per-brick sums of (z - zprev)^2
        for (int b = threadIdx.x; b < ndz; b += blockDim.x) acc[ST_DZ] += dzpart[b];
#pragma unroll
    for (int k = 0; k < ST_COUNT; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < ST_COUNT) {
        const int k = threadIdx.x;
        out[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

// ------------------------------------------------------------- warm start
// Algorithm 2 from a given z^0 and d^0 instead of zeros, in the reduced form:
// y^0 = V_r^T z^0 and w^0 = a.h - b.(y^0 - V_r^T d^0 / beta) (the f-step of
// Eq. DictVecSVD written for w, as the iteration carries it). One wave per voxel,
// lanes over the nodes q (coalesced reads of the voxel-major inputs): z^0 (and
// d^0 when dc is given, for the aux bracket) into the chunked state layout, the
// two contractions with V_r in float64 for NR ranks from NR blockIdx.y on,
// butterfly sums over the wave, then those rank rows below r of y and w (padded
// ranks keep their initial values; outside a mask everything stays as
// initialised, i.e. z = d = 0).
template <typename T, int NR>
__global__ void __launch_bounds__(256)
k_warm(IterArgs a, const double *__restrict__ z0, const double *__restrict__ d0,
       const double *__restrict__ V64, T *__restrict__ zc, T *__restrict__ dc, int Q) {
    const int lane = threadIdx.x & 63;
    const int64_t N = a.g.N;
    const int64_t n = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);   // one voxel per wave
    if (n >= N) return;
    if (a.code && (a.code[n] & 0x80u) == 0) return;
    const int r0 = NR * (int)blockIdx.y;
    double ya[NR], va[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) ya[i] = va[i] = 0.0;
    for (int q = lane; q < Q; q += 64) {
        const double zv = z0 ? z0[n * Q + q] : 0.0;
        const double dv = d0 ? d0[n * Q + q] : 0.0;
        if (blockIdx.y == 0) {
            const size_t e = ((size_t)(q / QC) * N + n) * QC + q % QC;
            zc[e] = (T)zv;
            if (dc) dc[e] = (T)dv;
        }
        const double *Vq = V64 + (size_t)q * a.RP + r0;
#pragma unroll
        for (int i = 0; i < NR; ++i)
            if (r0 + i < a.RP) {
                ya[i] += Vq[i] * zv;
                va[i] += Vq[i] * dv;
            }
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        ya[i] = wave_sum(ya[i]);
        va[i] = wave_sum(va[i]);
    }
    if (lane != 0) return;
    T *y = (T *)a.y, *w = (T *)a.w;
    const T *ah = (const T *)a.ah, *b = (const T *)a.bcoef;
#pragma unroll
    for (int i = 0; i < NR; ++i)
        if (r0 + i < a.r) {
            const size_t o = (size_t)(r0 + i) * N + n;
            y[o] = (T)ya[i];
            w[o] = (T)((double)ah[o] - (double)b[r0 + i] * (ya[i] - va[i] / a.beta));
        }
}

// ------------------------------------------------------------- output
template <typename T, typename O>
__global__ void __launch_bounds__(256)
k_output(const T *__restrict__ z, O *__restrict__ F, int Q, int64_t N) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * Q) return;
    const int64_t n = idx / Q;
    const int q = (int)(idx % Q);
    F[idx] = (O)z[chunk_index(q, n, N)];
}

// Four consecutive nodes per lane (Q % 4 == 0): a wave moves 4 voxels x 64 nodes,
// reading 256 contiguous bytes per chunk and writing 256 contiguous bytes per
// voxel row; block = 16 voxels, grid.y over groups of 64 nodes.
template <typename T, typename O>
__global__ void __launch_bounds__(256)
k_output4(const T *__restrict__ z, O *__restrict__ F, int Q, int64_t N) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t n = ((int64_t)blockIdx.x * 4 + wave) * 4 + (lane >> 4);
    const int q = (int)blockIdx.y * 64 + 4 * (lane & 15);
    if (n >= N || q >= Q) return;
    const T *src = z + chunk_index(q, n, N);     // q % 4 == 0: four nodes of one chunk
    O *dst = F + n * (int64_t)Q + q;
    if constexpr (sizeof(T) == 4 && sizeof(O) == 4) {
        *(float4 *)dst = *(const float4 *)src;
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) dst[i] = (O)src[i];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_zero(T *p, size_t count) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = (T)0;
}

// 16 bytes per lane (the bulk of a 16-byte aligned array)
__global__ void __launch_bounds__(256) k_zero16(uint4 *p, size_t count) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = uint4{0, 0, 0, 0};
}

__global__ void __launch_bounds__(256)
k_split_bf16(const float *__restrict__ V, uint16_t *__restrict__ hi, uint16_t *__restrict__ lo,
             size_t count) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float v = V[i];
    const float h = bf16_rne(v);
    const float l = bf16_rne(v - h);
    hi[i] = (uint16_t)(__float_as_uint(h) >> 16);
    lo[i] = (uint16_t)(__float_as_uint(l) >> 16);
}

inline unsigned blocks_for(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }

}  // namespace

// ------------------------------------------------------------- launchers
void launch_project(int mode, const void *M, int P, const double *Ur, const double *sig,
                    const double *acoef, int r, int RP, int64_t N, double *t, double *mperp2,
                    void *ah, void *w, void *y, int *bad, const uint8_t *code, hipStream_t s) {
    const dim3 grid(blocks_for(N, PJ_V)), block(256);
    if (mode == MODE_FP64)
        hipLaunchKernelGGL(k_project<MODE_FP64>, grid, block, 0, s, (const double *)M, P, Ur, sig,
                           acoef, r, RP, N, t, mperp2, (double *)ah, (double *)w, (double *)y, bad, code);
    else
        hipLaunchKernelGGL(k_project<MODE_FP32>, grid, block, 0, s, (const float *)M, P, Ur, sig,
                           acoef, r, RP, N, t, mperp2, (float *)ah, (float *)w, (float *)y, bad, code);
}

void launch_update_unfused(int mode, const IterArgs &a, hipStream_t s) {
    const dim3 grid(blocks_for(a.g.N * QC, 256), a.nchunk), block(256);
    if (mode == MODE_FP64) hipLaunchKernelGGL(k_update<MODE_FP64>, grid, block, 0, s, a);
    else if (mode == MODE_FP32) hipLaunchKernelGGL(k_update<MODE_FP32>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(k_update<MODE_BF16X3>, grid, block, 0, s, a);
}

void launch_projw_unfused(int mode, const IterArgs &a, hipStream_t s) {
    const dim3 grid(blocks_for(a.g.N, 256)), block(256);
    if (mode == MODE_FP64) hipLaunchKernelGGL((k_projw<MODE_FP64, 16>), grid, block, 0, s, a);
    else if (mode == MODE_FP32) hipLaunchKernelGGL((k_projw<MODE_FP32, 16>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_projw<MODE_BF16X3, 16>), grid, block, 0, s, a);
}

void launch_aux_pre(int mode, const IterArgs &a, void *t, void *f, const void *dprev,
                    hipStream_t s) {
    const dim3 grid(blocks_for(a.g.N * QC, 256), a.nchunk), block(256);
    if (mode == MODE_FP64)
        hipLaunchKernelGGL(k_aux_pre<MODE_FP64>, grid, block, 0, s, a, (double *)t, (double *)f,
                           (const double *)dprev);
    else if (mode == MODE_FP32)
        hipLaunchKernelGGL(k_aux_pre<MODE_FP32>, grid, block, 0, s, a, (float *)t, (float *)f,
                           (const float *)dprev);
    else
        hipLaunchKernelGGL(k_aux_pre<MODE_BF16X3>, grid, block, 0, s, a, (float *)t, (float *)f,
                           (const float *)dprev);
}

void launch_warm(int mode, const IterArgs &a, const double *z0, const double *d0, const double *V64,
                 void *zc, void *dc, int Q, hipStream_t s) {
    const dim3 grid(blocks_for(a.g.N, 4), a.RP <= 16 ? 1 : (a.RP + 31) / 32), block(256);
    if (mode == MODE_FP64) {
        if (a.RP <= 16)
            hipLaunchKernelGGL((k_warm<double, 16>), grid, block, 0, s, a, z0, d0, V64, (double *)zc,
                               (double *)dc, Q);
        else
            hipLaunchKernelGGL((k_warm<double, 32>), grid, block, 0, s, a, z0, d0, V64, (double *)zc,
                               (double *)dc, Q);
    } else {
        if (a.RP <= 16)
            hipLaunchKernelGGL((k_warm<float, 16>), grid, block, 0, s, a, z0, d0, V64, (float *)zc,
                               (float *)dc, Q);
        else
            hipLaunchKernelGGL((k_warm<float, 32>), grid, block, 0, s, a, z0, d0, V64, (float *)zc,
                               (float *)dc, Q);
    }
}

void launch_aux_post(int mode, void *t, const void *znew, double beta, size_t count,
                     hipStream_t s) {
    const dim3 grid(blocks_for((int64_t)count, 256)), block(256);
    if (mode == MODE_FP64)
        hipLaunchKernelGGL(k_aux_post<double>, grid, block, 0, s, (double *)t, (const double *)znew,
                           beta, count);
    else
        hipLaunchKernelGGL(k_aux_post<float>, grid, block, 0, s, (float *)t, (const float *)znew,
                           (float)beta, count);
}

// Blocks of the marching monitor that the current device runs at once (per CU
// occupancy x CUs), at most kMonitorBlocks; looked up once per device and build.
template <typename T, bool EXTRA>
int march_blocks() {
    static std::mutex mu;
    static int cache[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 1024;
    std::lock_guard<std::mutex> lk(mu);
    if (cache[dev] == 0) {
        int per = 0, cus = 0;
        const hipError_t e1 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_monitor_march<T, EXTRA>, 256, 0);
        const hipError_t e2 = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const int n = (e1 == hipSuccess && e2 == hipSuccess && per > 0 && cus > 0) ? per * cus : 1024;
        cache[dev] = std::min(n, kMonitorBlocks);
    }
    return cache[dev];
}

// Eight times the blocks per XCD: as few rounds of columns as the resident blocks
// allow, the XCD's run of columns spread evenly over them.
template <typename T, bool EXTRA>
int launch_march(const MonArgs &a, double *partial, hipStream_t s) {
    const int64_t ncol = ((a.g.nx + MT_X - 1) / MT_X) * ((a.g.ny + MT_Y - 1) / MT_Y) * a.nchunk;
    const int64_t cx = (ncol + 7) / 8, gmax = std::max(1, march_blocks<T, EXTRA>() / 8);
    const int64_t rounds = (cx + gmax - 1) / gmax, per = (cx + rounds - 1) / rounds;
    const int gx = (int)(8 * std::max<int64_t>(1, per));
    hipLaunchKernelGGL((k_monitor_march<T, EXTRA>), dim3(gx), dim3(256), 0, s, a, partial);
    return gx;
}

int monitor_blocks(int64_t N) {
    const int64_t b = ((N + 15) / 16 + 3) / 4;     // four 16-voxel tiles per block
    return (int)(b < kMonitorBlocks ? (b > 0 ? b : 1) : kMonitorBlocks);
}

void launch_monitor(int mode, const MonArgs &a, double *partial, double *out, hipStream_t s) {
    const int64_t esz = mode == MODE_FP64 ? 8 : 4;
    if (a.y && a.ld == 0 && a.yld == 0 && a.nchunk > 0 && a.nchunk <= kMonitorBlocks &&
        a.g.N * QC * esz + 64 < ((int64_t)1 << 31)) {
        // one pass along z: about as many blocks as the device runs at once (no tail)
        const bool extra = a.zprev || a.f || a.fstar;
        const int gx = mode == MODE_FP64 ? (extra ? launch_march<double, true>(a, partial, s)
                                                  : launch_march<double, false>(a, partial, s))
                                         : (extra ? launch_march<float, true>(a, partial, s)
                                                  : launch_march<float, false>(a, partial, s));
        hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, partial, gx, a.dzpart, a.ndz,
                           out);
        return;
    }
    // small grids with y given: one tile per block, the waves splitting chunks and ranks
    // (its loads go through 32-bit buffer offsets: the arrays must stay below 2^31 bytes)
    const int64_t ntile = (a.g.N + 15) / 16;
    const int64_t zbytes = (a.ld > 0 ? a.g.N * a.ld : (int64_t)a.nchunk * a.g.N * QC) * esz;
    const int64_t pbytes = a.ypart ? (int64_t)a.npart * a.RP * a.g.N * esz : 0;
    const bool sp = (a.y || a.ypart) && ntile <= kMonitorSpreadTiles && zbytes + 64 < ((int64_t)1 << 31) &&
                    pbytes + 64 < ((int64_t)1 << 31);
    const int nb = sp ? (int)(ntile > 0 ? ntile : 1) : monitor_blocks(a.g.N);
    const bool vm = a.ld > 0;
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(nb), dim3(256), 0, s, a, partial); };
    if (mode == MODE_FP64) {
        if (vm) sp ? go(k_monitor<double, true, true>) : go(k_monitor<double, true, false>);
        else sp ? go(k_monitor<double, false, true>) : go(k_monitor<double, false, false>);
    } else {
        if (vm) sp ? go(k_monitor<float, true, true>) : go(k_monitor<float, true, false>);
        else sp ? go(k_monitor<float, false, true>) : go(k_monitor<float, false, false>);
    }
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, partial, nb, a.dzpart, a.ndz, out);
}

void launch_output(int mode, const void *z, void *F, int Q, int64_t N, bool to_double,
                   hipStream_t s) {
    const bool aligned = ((reinterpret_cast<uintptr_t>(z) | reinterpret_cast<uintptr_t>(F)) & 15) == 0;
    if (Q % 4 == 0 && N > 0 && aligned && (N + 15) / 16 <= 0x7fffffff) {
        const dim3 grid4((unsigned)((N + 15) / 16), (unsigned)((Q + 63) / 64)), block4(256);
        if (mode == MODE_FP64)
            hipLaunchKernelGGL((k_output4<double, double>), grid4, block4, 0, s, (const double *)z,
                               (double *)F, Q, N);
        else if (to_double)
            hipLaunchKernelGGL((k_output4<float, double>), grid4, block4, 0, s, (const float *)z,
                               (double *)F, Q, N);
        else
            hipLaunchKernelGGL((k_output4<float, float>), grid4, block4, 0, s, (const float *)z,
                               (float *)F, Q, N);
        return;
    }
    const dim3 grid(blocks_for(N * Q, 256)), block(256);
    if (mode == MODE_FP64)
        hipLaunchKernelGGL((k_output<double, double>), grid, block, 0, s, (const double *)z,
                           (double *)F, Q, N);
    else if (to_double)
        hipLaunchKernelGGL((k_output<float, double>), grid, block, 0, s, (const float *)z,
                           (double *)F, Q, N);
    else
        hipLaunchKernelGGL((k_output<float, float>), grid, block, 0, s, (const float *)z,
                           (float *)F, Q, N);
}

void launch_zero(void *p, size_t count, int elem_bytes, hipStream_t s) {
    if (count == 0) return;
    const size_t bytes = count * (size_t)elem_bytes;
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0 && bytes >= 16 && bytes % 16 == 0) {
        const size_t n16 = bytes / 16;
        hipLaunchKernelGGL(k_zero16, dim3(blocks_for((int64_t)n16, 256)), dim3(256), 0, s, (uint4 *)p,
                           n16);
        return;
    }
    const dim3 grid(blocks_for((int64_t)count, 256)), block(256);
    if (elem_bytes == 8) hipLaunchKernelGGL(k_zero<double>, grid, block, 0, s, (double *)p, count);
    else if (elem_bytes == 4) hipLaunchKernelGGL(k_zero<float>, grid, block, 0, s, (float *)p, count);
    else hipLaunchKernelGGL(k_zero<uint16_t>, grid, block, 0, s, (uint16_t *)p, count);
}

void launch_split_bf16(const float *V, uint16_t *hi, uint16_t *lo, size_t count, hipStream_t s) {
    if (count == 0) return;
    hipLaunchKernelGGL(k_split_bf16, dim3(blocks_for((int64_t)count, 256)), dim3(256), 0, s, V,
                       hi, lo, count);
}

// ------------------------------------------------------------- allocation-free solves
// The device memory of an allocation-free solve: one file-scope array, which
// each device holds (at its own address) from the load of the library until
// the process ends. Host code never passes the array's name to a kernel: the
// name is a host-side stand-in, not a device address. The address of this
// device's copy is looked up once per device and kept.
namespace {
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_device_ptr(void **out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace ssmap
