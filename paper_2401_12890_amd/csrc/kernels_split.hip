// The LADMM iteration for small problems, split over spectral chunks.
//
// A grid with few bricks leaves most of the chip idle when each workgroup
// walks all Q nodes of its brick in turn (the fused kernel: a 32 x 32 grid is
// 8 bricks of 16 x 8). Here every (brick, 16-node chunk) pair is a workgroup
// of its own, so one launch has bricks x chunks workgroups. A workgroup
//   1. forms w^k for its brick's voxels from the r-vectors, with
//      y^k = sum over chunks of the partial products V_c^T z^k_c that the
//      previous launch left (added in chunk order, so results are repeatable):
//      w^k = a.h - b.(2 y^k - s^k), s^k = y^{k-1} + w^{k-1}  (s^0 = 0, w^0 = a.h),
//      the recursion w^k = a.h - b.(2 y^k - y^{k-1} - w^{k-1}) with one state
//      array instead of two;
//   2. stages z^k of its chunk (brick and one-voxel face halo) in LDS and
//      forms u = V_r w^k on the matrix cores (the f-step contraction of
//      Eq. DictVecSVD), the D^T D stencil of Eq. (l2) and the projected
//      z-update of Eq. (z2), and writes its chunk of z^{k+1};
//   3. writes its chunk's partial y^{k+1}_c = V_c^T z^{k+1}_c.
// The workgroup of chunk 0 also keeps s^{k+1} = y^k + w^k for the next launch. The
// r-vectors are double buffered by iteration parity, so no workgroup reads
// what another writes in the same launch. The lane mapping and the V operand
// blocks are those of the fused kernel (lane l: voxel l % 16 of a 16-voxel
// row, nodes 4 (l / 16) .. + 3 of the chunk).
#include "internal.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ssmap {

namespace {

typedef float v4f_s __attribute__((ext_vector_type(4)));
typedef double v4d_s __attribute__((ext_vector_type(4)));
typedef unsigned v4u_s __attribute__((ext_vector_type(4)));
typedef unsigned v2u_s __attribute__((ext_vector_type(2)));

template <int MODE> struct ST;
template <> struct ST<MODE_FP32> {
    using T = float;
    using V4 = v4f_s;
    static __device__ __forceinline__ V4 mfma(T a, T b, V4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ V4 load(__amdgpu_buffer_rsrc_t r, unsigned off) {
        return __builtin_bit_cast(V4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    }
    static __device__ __forceinline__ void store(V4 v, __amdgpu_buffer_rsrc_t r, unsigned off) {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4u_s, v), r, off, 0, 0);
    }
};
template <> struct ST<MODE_FP64> {
    using T = double;
    using V4 = v4d_s;
    typedef unsigned v8u __attribute__((ext_vector_type(8)));
    static __device__ __forceinline__ V4 mfma(T a, T b, V4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ V4 load(__amdgpu_buffer_rsrc_t r, unsigned off) {
        const v4u_s lo = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        const v4u_s hi = __builtin_amdgcn_raw_buffer_load_b128(r, off == kOOB ? kOOB : off + 16, 0, 0);
        return __builtin_bit_cast(V4, v8u{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]});
    }
    static __device__ __forceinline__ void store(V4 v, __amdgpu_buffer_rsrc_t r, unsigned off) {
        const v8u w = __builtin_bit_cast(v8u, v);
        __builtin_amdgcn_raw_buffer_store_b128(v4u_s{w[0], w[1], w[2], w[3]}, r, off, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b128(v4u_s{w[4], w[5], w[6], w[7]}, r,
                                               off == kOOB ? kOOB : off + 16, 0, 0);
    }
    static constexpr unsigned kOOB = 0x80000000u;
};

constexpr unsigned OOB = 0x80000000u;       // beyond every range: loads 0, stores dropped
constexpr int TX = 16;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, 0x00020000);
}

// Staged slots of a 16 x TY x TZ brick: the centre box, then its six face
// layers (halo edges and corners are never read). Slot -> halo-box coordinates.
template <int TY, int TZ> struct Slots {
    static constexpr int SX = TX + 2, SY = TY + 2, SZ = TZ + 2;
    static constexpr int C = TX * TY * TZ, XF = 2 * TY * TZ, YF = 2 * TX * TZ, ZF = 2 * TX * TY;
    static constexpr int NSLOT = C + XF + YF + ZF;
    static constexpr int NS = SX * SY * SZ;
    static constexpr int NSP = ((NS + 13) / 16) * 16 + 2;   // per-quad plane, 2 mod 16 entries
    static __device__ __forceinline__ void decode(int id, int &sx, int &sy, int &sz) {
        if (id < C) {
            sx = id % TX + 1;
            sy = (id / TX) % TY + 1;
            sz = id / (TX * TY) + 1;
            return;
        }
        id -= C;
        if (id < XF) {
            sx = (id & 1) ? TX + 1 : 0;
            sy = (id >> 1) % TY + 1;
            sz = (id >> 1) / TY + 1;
            return;
        }
        id -= XF;
        if (id < YF) {
            sx = id % TX + 1;
            sy = ((id / TX) & 1) ? TY + 1 : 0;
            sz = id / (2 * TX) + 1;
            return;
        }
        id -= YF;
        sx = id % TX + 1;
        sy = (id / TX) % TY + 1;
        sz = (id / (TX * TY)) ? TZ + 1 : 0;
    }
};

// KSU: u K-steps (ceil(r / 4)); RB: 16-rank blocks of the padded rank; TAIL:
// float32 ranks 17..20 with y of ranks 16..19 on the vector ALU (the operand
// blocks then carry one 16-rank y block and a tail table, as for the fused kernel).
// NT: threads (64 per 16-voxel row of the brick at most; 512 for the taller
// bricks, 256 and 128 for the 16 x 4 x 1 and 16 x 2 x 1 ones).
template <int MODE, int RB, int KSU, int TY, int TZ, int NT>
__global__ void __launch_bounds__(NT, 1)
k_split(SplitArgs sa, const TileRef *__restrict__ tiles) {
    using F = ST<MODE>;
    using T = typename F::T;
    using V4 = typename F::V4;
    using B = Slots<TY, TZ>;
    constexpr int NW = NT / 64;
    constexpr int NB = TY * TZ;
    constexpr int BPW = NB / NW;
    constexpr int NL = (4 * B::NSLOT + NT - 1) / NT;
    constexpr int KS = 4 * RB;
    constexpr bool TAIL = MODE == MODE_FP32 && RB == 2 && KSU == 5;
    constexpr int RBM = TAIL ? 1 : RB;
    constexpr int VB = (MODE == MODE_FP64 ? 4096 : 2048) * RB;   // bytes of a chunk's V block
    constexpr int PG = 8;                // chunk partials loaded per group
    static_assert(NB % NW == 0, "brick rows must split over the waves");
    // Thin bricks (at most 256 threads, registers to spare) keep the staged values in
    // registers until the row loads below have been issued too, so that both go out
    // in one memory round trip, and load their V operands straight into registers
    // (each lane's values are coalesced in the chunk's block); the 512-thread bricks
    // stage the block through LDS, which spares the registers.
    constexpr bool HOLD = NT <= 256;
    constexpr int VL = HOLD ? 1 : (VB / 16 + NT - 1) / NT;   // 16-byte pieces of the V block per thread
    static_assert(VB % 16 == 0, "V block of whole 16-byte pieces");
    __shared__ V4 lds[4 * B::NSP + 1];
    __shared__ uint4 ldsv[HOLD ? 1 : VB / 16];

    const IterArgs &a = sa.a;
    // One argument from each 64-byte line of the argument block, needed together:
    // all four lines arrive in one scalar round trip, and the argument loads the
    // compiler places later (after the brick lookup) hit the scalar cache instead
    // of waiting out a miss just before the first vector load. (An empty asm
    // statement: it only asks for the values in scalar registers at this point.)
    asm volatile("" ::"s"(a.z), "s"(a.nchunk), "s"(a.code), "s"(sa.sout));
    const int nch = a.nchunk;
    // Workgroup b runs on XCD b % 8. Each XCD takes one contiguous eighth of the
    // brick-major (brick, chunk) list, so the chunk workgroups of a brick, which all
    // read the brick's y partials and r-vectors, share one L2 and its write-backs.
    const int item = [] {
        const int total = (int)gridDim.x, b = (int)blockIdx.x, x = b & 7;
        return x * (total >> 3) + min(x, total & 7) + (b >> 3);
    }();
    // the brick: from the table for a masked grid (only bricks with an inside
    // voxel), else straight from the index (x-fastest order, as the table lists it)
    TileRef tr;
    if (a.code) {
        tr = tiles[item / nch];
    } else {
        const int bi = item / nch;
        const int bx = (int)((a.g.nx + TX - 1) / TX), byc = (int)((a.g.ny + TY - 1) / TY);
        tr = TileRef{0, bi % bx, (bi / bx) % byc, bi / (bx * byc)};
    }
    const int c = item % nch;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = lane & 15, i4 = lane >> 4;
    const int64_t nx = a.g.nx, ny = a.g.ny, nz = a.g.nz, N = a.g.N;
    const int64_t x0 = (int64_t)tr.tx * TX, y0 = (int64_t)tr.ty * TY, z0 = (int64_t)tr.tz * TZ;
    const size_t chunk_elems = (size_t)N * QC;
    const unsigned chunk_bytes = (unsigned)(chunk_elems * sizeof(T));
    const T tau = (T)a.tau, lam2 = (T)a.lam2, beta = (T)a.beta;

    // ---- stage z^k of chunk c (brick and face halo) and, for the 512-thread bricks,
    // the chunk's V operand block
    V4 R[NL];
    int loff[NL];
    uint4 Rv[VL];
    auto stage_to_lds = [&]() {
#pragma unroll
        for (int l = 0; l < NL; ++l) lds[loff[l]] = R[l];
        if constexpr (!HOLD)
#pragma unroll
            for (int v = 0; v < VL; ++v)
                if (tid + NT * v < VB / 16) ldsv[tid + NT * v] = Rv[v];
    };
    {
        const __amdgpu_buffer_rsrc_t zr = rsrc((const T *)a.z + (size_t)c * chunk_elems, chunk_bytes);
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const int f = tid + NT * l;
            unsigned off = OOB;
            loff[l] = 4 * B::NSP;        // sink entry for unused lanes
            if (f < 4 * B::NSLOT) {
                int sx, sy, sz;
                B::decode(f >> 2, sx, sy, sz);
                loff[l] = (f & 3) * B::NSP + sx + B::SX * (sy + B::SY * sz);
                const int64_t gx = x0 + sx - 1, gy = y0 + sy - 1, gz = z0 + sz - 1;
                if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz)
                    off = (unsigned)(((gx + nx * (gy + ny * gz)) * QC + 4 * (f & 3)) * sizeof(T));
            }
            R[l] = F::load(zr, off);
        }
        if constexpr (!HOLD) {
            const __amdgpu_buffer_rsrc_t vr = rsrc(a.Vu, (unsigned)(nch * VB));
#pragma unroll
            for (int v = 0; v < VL; ++v) {
                const int piece = tid + NT * v;
                Rv[v] = __builtin_bit_cast(
                    uint4, __builtin_amdgcn_raw_buffer_load_b128(
                               vr, piece < VB / 16 ? (unsigned)(c * VB + 16 * piece) : OOB, 0, 0));
            }
            stage_to_lds();
        }
    }

    // ---- V operands of the chunk: lane l takes element e * 64 + l of the block for
    // the u steps and the y blocks, and the tail table of its quad (float32 ranks 17..20)
    T vu[KSU], vy[RBM][4], vt[TAIL ? 4 : 1][4];
    auto v_operands = [&](auto &&elem) {
#pragma unroll
        for (int s = 0; s < KSU; ++s) vu[s] = elem(s * 64 + lane);
#pragma unroll
        for (int rb = 0; rb < RBM; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) vy[rb][i] = elem((KS + rb * 4 + i) * 64 + lane);
        if constexpr (TAIL) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int t = 0; t < 4; ++t) vt[i][t] = elem((KS + 4) * 64 + i4 * 16 + i * 4 + t);
        }
    };
    if constexpr (HOLD) {                // issued with the row loads below
        const __amdgpu_buffer_rsrc_t vr = rsrc(a.Vu, (unsigned)(nch * VB));
        v_operands([&](int e) -> T {
            const unsigned off = (unsigned)(c * VB) + (unsigned)(e * sizeof(T));
            if constexpr (sizeof(T) == 8)
                return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(vr, off, 0, 0));
            else
                return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(vr, off, 0, 0));
        });
    }

    // ---- per-row voxels and w^k of the u operand (lane: ranks 4 s + l/16, voxel j)
    int64_t nvox[BPW];
    bool valid[BPW], inside[BPW];
    T deg[BPW];
    unsigned soff[BPW];
    T wop[BPW][KSU];
    const size_t pstride = (size_t)a.RP * N;
    const unsigned pbytes1 = (unsigned)(pstride * sizeof(T));      // one chunk's partials
    const __amdgpu_buffer_rsrc_t prs = rsrc(sa.pin, (unsigned)(nch * (size_t)pbytes1)),
                                 sir = rsrc(sa.sin, pbytes1), sor = rsrc(sa.sout, pbytes1),
                                 ahr = rsrc(a.ah, pbytes1),
                                 bcr = rsrc(a.bcoef, (unsigned)(a.RP * sizeof(T)));
    auto ld1 = [](const __amdgpu_buffer_rsrc_t &r, unsigned off) -> T {
        if constexpr (sizeof(T) == 8)
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
        else
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    };
    auto st1 = [](T v, const __amdgpu_buffer_rsrc_t &r, unsigned off) {
        if constexpr (sizeof(T) == 8)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u_s, v), r, off, 0, 0);
        else
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
    };
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
        const int row = wave + NW * b;
        const int by = row % TY, bz = row / TY;
        const int64_t gx = x0 + j, gy = y0 + by, gz = z0 + bz;
        valid[b] = gx < nx && gy < ny && gz < nz;
        nvox[b] = valid[b] ? gx + nx * (gy + ny * gz) : 0;
        deg[b] = (T)((gx > 0) + (gx + 1 < nx) + (gy > 0) + (gy + 1 < ny) + (gz > 0) + (gz + 1 < nz));
        inside[b] = valid[b];
        if (a.code) {
            const unsigned cb = a.code[nvox[b]];
            deg[b] = (T)(cb & 7u);
            inside[b] = valid[b] && (cb & 0x80u) != 0;
        }
        soff[b] = valid[b] ? (unsigned)((nvox[b] * QC + 4 * i4) * sizeof(T)) : OOB;
        // y^k of the lane's ranks: the chunks' partials added in chunk order. All
        // loads of a group of PG chunks issue before any addition (out-of-range
        // chunks and ranks read 0, which leaves the sums unchanged).
        unsigned orr[KSU];
        T yk[KSU], ahv[KSU], bcv[KSU], siv[KSU];
#pragma unroll
        for (int s = 0; s < KSU; ++s) {
            const int rr = 4 * s + i4;
            orr[s] = rr < a.r && valid[b] ? (unsigned)(((size_t)rr * N + nvox[b]) * sizeof(T)) : OOB;
            yk[s] = (T)0;
            ahv[s] = ld1(ahr, orr[s]);   // issued with the partials below
            bcv[s] = ld1(bcr, rr < a.r ? (unsigned)(rr * sizeof(T)) : OOB);
            siv[s] = ld1(sir, orr[s]);
        }
        for (int c0 = 0; c0 < nch; c0 += PG) {
            T pv[PG][KSU];
#pragma unroll
            for (int u = 0; u < PG; ++u)
#pragma unroll
                for (int s = 0; s < KSU; ++s)
                    pv[u][s] = ld1(prs, c0 + u < nch && orr[s] != OOB
                                            ? (unsigned)((c0 + u) * pbytes1) + orr[s] : OOB);
#pragma unroll
            for (int u = 0; u < PG; ++u)
#pragma unroll
                for (int s = 0; s < KSU; ++s) yk[s] += pv[u][s];
        }
#pragma unroll
        for (int s = 0; s < KSU; ++s) {
            const T wk = ahv[s] - bcv[s] * ((T)2 * yk[s] - siv[s]);
            wop[b][s] = wk;
            if (c == 0) {                // kept for the next launch
                st1(yk[s] + wk, sor, orr[s]);
            }
        }
    }
    if constexpr (HOLD) stage_to_lds();
    __syncthreads();

    // ---- the update of the chunk's 16 nodes, partial y^{k+1}
    if constexpr (!HOLD) v_operands([&](int e) -> T { return ((const T *)ldsv)[e]; });
    const __amdgpu_buffer_rsrc_t zo = rsrc((T *)a.znew + (size_t)c * chunk_elems, chunk_bytes);
    const unsigned pbytes = (unsigned)(pstride * sizeof(T));
    const __amdgpu_buffer_rsrc_t po = rsrc((T *)sa.pout + (size_t)c * pstride, pbytes);
    const V4 *L = lds + i4 * B::NSP;
    constexpr int SZ = B::SX * B::SY;
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
        V4 u = V4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KSU; ++s) u = F::mfma(vu[s], wop[b][s], u);
        const int row = wave + NW * b;
        const int sl = (j + 1) + B::SX * ((row % TY + 1) + B::SY * (row / TY + 1));
        const V4 zc = L[sl];
        const V4 nsum = (L[sl - 1] + L[sl + 1]) + (L[sl - B::SX] + L[sl + B::SX]) +
                        (L[sl - SZ] + L[sl + SZ]);
        const V4 lap = deg[b] * zc - nsum;
        V4 zn = zc - tau * (lam2 * lap - beta * u);
#pragma unroll
        for (int i = 0; i < 4; ++i) zn[i] = (zn[i] > (T)0 && inside[b]) ? zn[i] : (T)0;
        F::store(zn, zo, soff[b]);
        // partial y^{k+1} of this chunk: K-row l/16 of step i is node 4 (l/16) + i
        V4 yacc[RBM];
#pragma unroll
        for (int rb = 0; rb < RBM; ++rb) {
            yacc[rb] = V4{0, 0, 0, 0};
#pragma unroll
            for (int i = 0; i < 4; ++i) yacc[rb] = F::mfma(vy[rb][i], zn[i], yacc[rb]);
        }
        T ytail[4] = {(T)0, (T)0, (T)0, (T)0};
        if constexpr (TAIL) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
#pragma unroll
                for (int i = 0; i < 4; ++i) ytail[t] += vt[i][t] * zn[i];
                ytail[t] += __shfl_xor(ytail[t], 16);
                ytail[t] += __shfl_xor(ytail[t], 32);
            }
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // f64 16x16x4 returns rows l/16 + 4 i; f32 rows 4 (l/16) + i
                const int rr = MODE == MODE_FP64 ? 16 * rb + i4 + 4 * i : 16 * rb + 4 * i4 + i;
                T yv;
                if constexpr (TAIL) yv = rb == 0 ? yacc[0][i] : ytail[i];
                else yv = yacc[rb][i];
                const unsigned ob = rr < a.r && valid[b] ? (unsigned)(((size_t)rr * N + nvox[b]) * sizeof(T)) : OOB;
                if constexpr (sizeof(T) == 8)
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u_s, yv), po, ob, 0, 0);
                else
                    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, yv), po, ob, 0, 0);
            }
    }
}

template <int MODE, int RB, int KSU, int TY, int TZ, int NT = 512>
void launch_s(const SplitArgs &sa, const TileRef *tiles, int ntiles, hipStream_t s) {
    hipLaunchKernelGGL((k_split<MODE, RB, KSU, TY, TZ, NT>), dim3(ntiles * sa.a.nchunk), dim3(NT), 0, s,
                       sa, tiles);
}

template <int MODE, int RB, int KSU>
bool split_shape(const SplitArgs &sa, FusedShape sh, const TileRef *tiles, int ntiles, hipStream_t s) {
    if (sh.ty == 2 && sh.tz == 1) return launch_s<MODE, RB, KSU, 2, 1, 128>(sa, tiles, ntiles, s), true;
    if (sh.ty == 4 && sh.tz == 1) return launch_s<MODE, RB, KSU, 4, 1, 256>(sa, tiles, ntiles, s), true;
    if (sh.ty == 8 && sh.tz == 1) return launch_s<MODE, RB, KSU, 8, 1>(sa, tiles, ntiles, s), true;
    if (sh.ty == 16 && sh.tz == 1) return launch_s<MODE, RB, KSU, 16, 1>(sa, tiles, ntiles, s), true;
    if (sh.ty == 4 && sh.tz == 2) return launch_s<MODE, RB, KSU, 4, 2>(sa, tiles, ntiles, s), true;
    if (sh.ty == 4 && sh.tz == 4) return launch_s<MODE, RB, KSU, 4, 4>(sa, tiles, ntiles, s), true;
    if (sh.ty == 8 && sh.tz == 4) return launch_s<MODE, RB, KSU, 8, 4>(sa, tiles, ntiles, s), true;
    return false;
}

template <int MODE>
bool split_mode(const SplitArgs &sa, FusedShape sh, const TileRef *tiles, int ntiles, hipStream_t s) {
    const int r = sa.a.r;
    if (r <= 16) return split_shape<MODE, 1, 4>(sa, sh, tiles, ntiles, s);
    if (r <= 20) return split_shape<MODE, 2, 5>(sa, sh, tiles, ntiles, s);
    if (r <= 24) return split_shape<MODE, 2, 6>(sa, sh, tiles, ntiles, s);
    return split_shape<MODE, 2, 8>(sa, sh, tiles, ntiles, s);
}

}  // namespace

bool launch_split(int mode, const SplitArgs &sa, FusedShape sh, const TileRef *tiles, int ntiles,
                  hipStream_t s) {
    if (ntiles <= 0) return true;
    if (mode == MODE_FP64) return split_mode<MODE_FP64>(sa, sh, tiles, ntiles, s);
    if (mode == MODE_FP32) return split_mode<MODE_FP32>(sa, sh, tiles, ntiles, s);
    return false;
}

}  // namespace ssmap
