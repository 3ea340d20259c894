// Fused single-pass LADMM iteration with MFMA contractions (gfx950).
//
// One workgroup owns a brick of TX x TY x TZ voxels (TX = 16) and streams
// all Q spectral nodes of it in chunks of 16. Per chunk it
//   1. stages z^k of the brick and its one-voxel face halo into LDS,
//   2. forms u = V_r w^k on the matrix cores (the f-step contraction of
//      Eq. DictVecSVD, M = 16 nodes, N = 16 voxels, K = r),
//   3. applies the D^T D stencil of Eq. (l2) on every plane of the chunk
//      from LDS, the linearised z-update of Eq. (z2) and the projection onto
//      z >= 0, and writes z^{k+1},
//   4. accumulates y^{k+1} = V_r^T z^{k+1} on the matrix cores
//      (M = 16 ranks, N = 16 voxels, K = 16 nodes), straight from the
//      registers that hold z^{k+1}.
// After the last chunk each voxel's r-vectors are updated
// (w^{k+1} = a.h - b.(2 y^{k+1} - y^k - w^k)). z is read once from HBM
// and written once per iteration; f and d never touch HBM.
//
// Lane mapping (64-lane wave, 16x16 MFMA output): lane l holds voxel
// j = l % 16 of a 16-voxel row and the four consecutive nodes
// 4*(l/16) .. 4*(l/16)+3 of the chunk. That is exactly the MFMA D layout,
// so u arrives where the stencil needs it, and z^{k+1} is fed back as the
// B operand of the second contraction by permuting the contraction index
// (step i uses node 4*(l/16)+i in K-row l/16), with V's A operand
// permuted the same way when it is prepared on the host.
#include "internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>

namespace ssmap {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

typedef short v4s __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

// bf16 bits of a float, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned bf16_bits(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_val(unsigned bits) { return __uint_as_float(bits << 16); }

// hi/lo bf16 split of 4 floats into two short4 operands
__device__ __forceinline__ void split4(const v4f &x, v4s &hi, v4s &lo) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const unsigned h = bf16_bits(x[i]);
        hi[i] = (short)h;
        lo[i] = (short)bf16_bits(x[i] - bf16_val(h));
    }
}

template <int MODE> struct FT;
template <> struct FT<MODE_BF16X3> {
    using T = float;
    using V4 = v4f;
};
template <> struct FT<MODE_FP32> {
    using T = float;
    using V4 = v4f;
    static __device__ __forceinline__ V4 mfma(T a, T b, V4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct FT<MODE_FP64> {
    using T = double;
    using V4 = v4d;
    static __device__ __forceinline__ V4 mfma(T a, T b, V4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

constexpr int TX = 16;

// Slots of the staged brick: the centre box plus the six one-voxel face
// layers (edges and corners of the halo box are never read).
template <int TY, int TZ> struct Brick {
    static constexpr int SX = TX + 2, SY = TY + 2, SZ = TZ + 2;
    static constexpr int NS = SX * SY * SZ;
    // per-quad plane padded to 2 mod 16 entries: the staging stores (the four
    // quads of two adjacent slots per eight lanes) fall on distinct banks; this
    // halved the measured LDS bank-conflict cycles against 4 mod 16
    static constexpr int NSP = ((NS + 13) / 16) * 16 + 2;
    static constexpr int C = TX * TY * TZ;
    static constexpr int XF = 2 * TY * TZ;
    static constexpr int YF = 2 * TX * TZ;
    static constexpr int ZF = 2 * TX * TY;
    static constexpr int NSLOT = C + XF + YF + ZF;

    // staged slot id -> halo-box coordinates (0..SX-1, ...)
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

// Bytes of the per-chunk V operand block (u operand image, then y operand image).
template <int MODE, int RB> struct VopSize {
    static constexpr int bytes = MODE == MODE_BF16X3 ? 2048 + 1024 * RB
                               : (MODE == MODE_FP64 ? 4096 * RB : 2048 * RB);
};

constexpr int NT = 512;                 // threads per workgroup (8 waves)
constexpr unsigned OOB = 0x80000000u;   // buffer offset beyond every range: loads 0, stores dropped
constexpr int RSRC_W3 = 0x00020000;     // buffer descriptor word 3 (raw buffer, gfx9 family)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, RSRC_W3);
}

// Neighbour along x inside a 16-lane row by DPP: lane j takes lane j - 1
// (SHR) or j + 1 (SHL) of its row; the lane at the row's edge keeps `edge`.
template <bool SHR>
__device__ __forceinline__ unsigned dpp_x(unsigned edge, unsigned v) {
    return (unsigned)__builtin_amdgcn_update_dpp((int)edge, (int)v, SHR ? 0x111 : 0x101, 0xF, 0xF,
                                                 false);
}
template <bool SHR>
__device__ __forceinline__ v4f dpp_x(v4f edge, v4f v) {
    v4f o;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        o[k] = __uint_as_float(dpp_x<SHR>(__float_as_uint(edge[k]), __float_as_uint(v[k])));
    return o;
}

// Four state values (16 B for float, 32 B for double) through a buffer resource.
// Stores of z^{k+1} are non-temporal (CPol NT): nothing reads them again in this
// launch (measured 4 % faster); loads stay cached, so a face halo that a brick
// running at the same time on the same XCD has just loaded can hit its L2.
constexpr int NT_STORE = 2;
template <typename T, typename V4> struct Buf;
template <> struct Buf<float, v4f> {
    static __device__ __forceinline__ v4f load(__amdgpu_buffer_rsrc_t r, unsigned off) {
        return __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    }
    static __device__ __forceinline__ void store(v4f v, __amdgpu_buffer_rsrc_t r, unsigned off) {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4u, v), r, off, 0, NT_STORE);
    }
};
template <> struct Buf<double, v4d> {
    typedef unsigned v8u __attribute__((ext_vector_type(8)));
    static __device__ __forceinline__ v4d load(__amdgpu_buffer_rsrc_t r, unsigned off) {
        const v4u lo = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        const v4u hi = __builtin_amdgcn_raw_buffer_load_b128(r, off == OOB ? OOB : off + 16, 0, 0);
        const v8u w = v8u{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        return __builtin_bit_cast(v4d, w);
    }
    static __device__ __forceinline__ void store(v4d v, __amdgpu_buffer_rsrc_t r, unsigned off) {
        const v8u w = __builtin_bit_cast(v8u, v);
        __builtin_amdgcn_raw_buffer_store_b128(v4u{w[0], w[1], w[2], w[3]}, r, off, 0, NT_STORE);
        __builtin_amdgcn_raw_buffer_store_b128(v4u{w[4], w[5], w[6], w[7]}, r,
                                               off == OOB ? OOB : off + 16, 0, NT_STORE);
    }
};

// Monitored iterations: the brick's sum of (z^{k+1} - z^k)^2 (float64) over the
// waves, written to mon[tile] (one slot per brick, summed in a fixed order later).
__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}
template <int NW>
__device__ __forceinline__ void brick_sum_out(double v, double *red, double *mon, int tile) {
    v = wave_sum64(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += red[w];
        mon[tile] = t;
    }
}

// KSU: K-steps of the u contraction actually needed (ceil(r / 4)); RB: 16-row
// blocks of r in the y contraction. bf16x3 uses one 32-wide K-step (KSU unused).
// Small volumetric bricks (16 x 4 x 4: two rows per wave) of the float32 and
// bf16x3 register-staged kernel are built for four waves per SIMD, i.e. two
// workgroups per CU (measured faster there); the others keep the registers
// they need (measured: capping planar bricks at 128 registers spills).
constexpr bool fused_small(int mode, int ty, int tz) {
    return mode != MODE_FP64 && tz > 1 && ty * tz <= 16;
}
constexpr int fused_occupancy(int mode, int ty, int tz) { return fused_small(mode, ty, tz) ? 4 : 1; }

template <int MODE, int RB, int KSU, int TY, int TZ, bool MON>
__global__ void __launch_bounds__(NT, fused_occupancy(MODE, TY, TZ))
k_fused(const IterArgs *__restrict__ jobs, const TileRef *__restrict__ tiles, int ntiles,
        int round, double *__restrict__ mon) {
    using F = FT<MODE>;
    using T = typename F::T;
    using V4 = typename F::V4;
    using B = Brick<TY, TZ>;
    using IO = Buf<T, V4>;
    constexpr bool BF = MODE == MODE_BF16X3;
    constexpr int NW = NT / 64;
    constexpr int NB = TY * TZ;          // 16-voxel rows in the brick
    constexpr int BPW = NB / NW;         // rows per wave
    constexpr int NL = (4 * B::NSLOT + NT - 1) / NT;   // staged quads per thread
    constexpr int VB = VopSize<MODE, RB>::bytes;
    constexpr int KS = 4 * RB;           // stride of the u part of the V block
    // ranks 17..20: y of ranks 16..19 on the vector ALU (16 FMAs per row and
    // chunk) instead of a second, mostly padded 16-rank MFMA block
    constexpr bool TAIL = MODE == MODE_FP32 && RB == 2 && KSU == 5;
    constexpr int RBM = TAIL ? 1 : RB;   // 16-rank blocks on the matrix cores
    static_assert(NB % NW == 0, "brick rows must split over the waves");
    static_assert(VB % 16 == 0 && VB / 16 <= NT, "V operand block must stage in one pass");
    static_assert(BF || (KSU >= 1 && KSU <= KS), "u K-steps must fit the padded rank");

    // The float32 16 x 8 x 4 and 16 x 16 x 1 and the float64 16 x 8 x 1 and
    // 16 x 4 x 2 bricks double-buffer their LDS (one workgroup per CU): chunk c + 1 is stored while
    // chunk c is read, one barrier per chunk, the loads two chunks ahead (float32
    // planar: 10 % faster on the batched slices than two single-buffered
    // workgroups per CU). For short spectra they also run persistent: a workgroup
    // takes several bricks in turn and the loads of a brick's first chunks overlap
    // the end of the one before it.
    constexpr bool DBL = (MODE == MODE_FP32 && ((TY == 8 && TZ == 4) || (TY == 16 && TZ == 1))) ||
                         (MODE == MODE_FP64 && ((TY == 8 && TZ == 1) || (TY == 4 && TZ == 2)));
    constexpr int NBUF = DBL ? 2 : 1;
    __shared__ V4 lds[NBUF][4 * B::NSP + 1];   // z^k of the brick, [quad][slot], + one sink entry
    __shared__ uint4 ldsv[NBUF][NT];           // V operands of the chunk (entries >= VB/16 unused)
    __shared__ double mred[MON ? NW : 1];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int j = lane & 15;
    const int i4 = lane >> 4;

    // ---- bricks of this workgroup. For short spectra the double-buffered bricks
    //      run a persistent grid (about one workgroup per CU, each taking its
    //      bricks in turn); otherwise every workgroup takes one brick. Either way
    //      the bricks of an XCD form one contiguous run of the table (neighbours
    //      share its L2).
    auto tile_of = [&](int it) -> int {  // it-th brick of this workgroup, -1 past the last
        const int b = blockIdx.x, nwg = gridDim.x;
        if ((ntiles & 7) == 0 && (nwg & 7) == 0) {
            const int per = ntiles >> 3, k = (b >> 3) + it * (nwg >> 3);
            return k < per ? (b & 7) * per + k : -1;
        }
        const int k = b + it * nwg;
        return k < ntiles ? k : -1;
    };
    // two descriptors per job (z^k -> z^{k+1} for even and odd k); a job that
    // joined a shared loop late carries its phase
    auto args_of = [&](int tile) -> const IterArgs & {
        const int job = tiles[tile].job;
        return jobs[2 * job + ((round + jobs[2 * job].phase) & 1)];
    };

    // ---- LDS entry of each quad this thread stages (the sink for unused lanes),
    //      the same for every brick
    int loff[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const int f = tid + NT * l;
        loff[l] = 4 * B::NSP;
        if (f < 4 * B::NSLOT) {
            int sx, sy, sz;
            B::decode(f >> 2, sx, sy, sz);
            loff[l] = (f & 3) * B::NSP + sx + B::SX * (sy + B::SY * sz);
        }
    }

    // ---- the load stream: one fetch brings the z quads and the V operand block of
    //      one chunk into registers. With a double-buffered shape a workgroup
    //      streams chunk 0 .. nchunk-1 of each of its bricks in turn (past the last
    //      brick every offset is out of range: zeros, no memory traffic); the other
    //      shapes re-read their last chunk at the end (one loop path with exact
    //      wait counts).
    V4 R[NL];
    uint4 Rv;
    unsigned voff[NL];                   // byte offset of the staged quad in a chunk (OOB: zero)
    const T *fz = nullptr;
    const void *fv = nullptr;
    size_t fce = 0;                      // elements of a z chunk
    unsigned fcb = 0, fvb = 0;           // bytes of a z chunk, of all V operand blocks
    int fit = 0, fc = 0, fn = 0;         // brick ordinal, chunk, chunks of that brick
    const unsigned vlane = tid < VB / 16 ? (unsigned)tid * 16 : OOB;
    auto fseek = [&](int it) {           // the stream to chunk 0 of the it-th brick
        const int t = tile_of(it);
        fit = it;
        fc = fn = 0;
        fce = 0;
        fcb = fvb = 0;
        int64_t gx0 = 0, gy0 = 0, gz0 = 0, mx = 0, my = 0, mz = 0;
        if (t >= 0) {
            const IterArgs &fa = args_of(t);
            const TileRef ft = tiles[t];
            fz = (const T *)fa.z;
            fv = fa.Vu;
            fce = (size_t)fa.g.N * QC;
            fcb = (unsigned)(fce * sizeof(T));
            fvb = (unsigned)(fa.nchunk * VB);
            fn = fa.nchunk;
            mx = fa.g.nx;
            my = fa.g.ny;
            mz = fa.g.nz;
            gx0 = (int64_t)ft.tx * TX - 1;
            gy0 = (int64_t)ft.ty * TY - 1;
            gz0 = (int64_t)ft.tz * TZ - 1;
        }
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const int f = tid + NT * l;
            voff[l] = OOB;
            if (f < 4 * B::NSLOT) {
                int sx, sy, sz;
                B::decode(f >> 2, sx, sy, sz);
                const int64_t gx = gx0 + sx, gy = gy0 + sy, gz = gz0 + sz;
                if (gx >= 0 && gx < mx && gy >= 0 && gy < my && gz >= 0 && gz < mz)
                    voff[l] = (unsigned)(((gx + mx * (gy + my * gz)) * QC + 4 * (f & 3)) * sizeof(T));
            }
        }
    };
    auto fetch = [&]() {
        const __amdgpu_buffer_rsrc_t zr = rsrc(fz + (size_t)fc * fce, fcb), vr = rsrc(fv, fvb);
        Rv = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                           vr, vlane == OOB ? OOB : vlane + (unsigned)(fc * VB), 0, 0));
#pragma unroll
        for (int l = 0; l < NL; ++l) R[l] = IO::load(zr, voff[l]);
        if (++fc == fn) {
            if constexpr (DBL)
                fseek(fit + 1);
            else
                fc = fn - 1;
        }
    };
    auto stage = [&](int buf) {          // registers -> LDS (out-of-grid slots hold zeros)
#pragma unroll
        for (int l = 0; l < NL; ++l)     // unused staging lanes (whole waves) store nothing
            if (NT * (l + 1) <= 4 * B::NSLOT || tid + NT * l < 4 * B::NSLOT) lds[buf][loff[l]] = R[l];
        ldsv[buf][tid] = Rv;
    };
    fseek(0);
    fetch();
    if constexpr (DBL) {
        stage(0);
        fetch();
        __syncthreads();
    }

    // ---- halo-box slot of this lane's voxel in each of its rows (any brick)
    int slot0[BPW];
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
        const int row = wave + NW * b;
        slot0[b] = (j + 1) + B::SX * ((row % TY + 1) + B::SY * (row / TY + 1));
    }

    int g = 0;                           // chunks computed so far (LDS buffer parity)
    T dzacc = 0;                         // monitored iterations: this lane's sum of
                                         // (z^{k+1} - z^k)^2 over a brick (state type)
    for (int it = 0;; ++it) {
        const int tile = tile_of(it);
        if (tile < 0) break;
        const bool more = tile_of(it + 1) >= 0;   // the stream runs on into a next brick
        const TileRef tr = tiles[tile];
        const IterArgs &a = args_of(tile);
        const int64_t nx = a.g.nx, ny = a.g.ny, nz = a.g.nz, N = a.g.N;
        const int64_t x0 = (int64_t)tr.tx * TX, y0 = (int64_t)tr.ty * TY, z0 = (int64_t)tr.tz * TZ;
        const T tau = (T)a.tau, lam2 = (T)a.lam2, beta = (T)a.beta;
        const size_t chunk_elems = (size_t)N * QC;
        const unsigned chunk_bytes = (unsigned)(chunk_elems * sizeof(T));

        // ---- per-row voxel coordinates, neighbour count and store offsets
        int64_t nvox[BPW];
        bool valid[BPW];
        T deg[BPW];
        bool inside[BPW];                // false: outside a mask (z stays 0)
        unsigned soff[BPW];              // byte offset of this lane's quad in a chunk
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
            const int row = wave + NW * b;
            const int by = row % TY, bz = row / TY;
            const int64_t gx = x0 + j, gy = y0 + by, gz = z0 + bz;
            valid[b] = gx < nx && gy < ny && gz < nz;
            nvox[b] = valid[b] ? gx + nx * (gy + ny * gz) : 0;
            deg[b] = (T)((gx > 0) + (gx + 1 < nx) + (gy > 0) + (gy + 1 < ny) + (gz > 0) + (gz + 1 < nz));
            inside[b] = valid[b];        // lanes beyond the grid compute z^{k+1} = 0 (never stored)
            if (a.code) {                // masked grid: outside voxels hold z = 0, so the
                const unsigned cb = a.code[nvox[b]];   // box neighbour sum stays exact
                deg[b] = (T)(cb & 7u);
                inside[b] = valid[b] && (cb & 0x80u) != 0;
            }
            soff[b] = valid[b] ? (unsigned)((nvox[b] * QC + 4 * i4) * sizeof(T)) : OOB;
        }

        // ---- B operand of u = V_r w. fp32/fp64: lane holds w[r = 4 s + l/16][voxel j];
        //      bf16x3: lane holds w[r = 8 (l/16) + jj][voxel j], jj < 8, split hi/lo.
        const T *wsrc = (const T *)a.w;
        T wop[BPW][BF ? 1 : KSU];
        v8bf whi[BF ? BPW : 1], wlo[BF ? BPW : 1];
        V4 yacc[BPW][RBM];
        T ytail[TAIL ? BPW : 1][4];      // partial y of ranks 16..19 over this lane's nodes
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
#pragma unroll
            for (int t = 0; t < 4; ++t) ytail[TAIL ? b : 0][t] = (T)0;
            if constexpr (BF) {
                v4u h = v4u{0, 0, 0, 0}, l = v4u{0, 0, 0, 0};
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) {
                    const int r = 8 * i4 + jj;
                    const float v = r < a.RP ? wsrc[(size_t)r * N + nvox[b]] : 0.0f;
                    const unsigned hb = bf16_bits(v);
                    const unsigned lb = bf16_bits(v - bf16_val(hb));
                    h[jj >> 1] |= hb << (16 * (jj & 1));
                    l[jj >> 1] |= lb << (16 * (jj & 1));
                }
                whi[b] = __builtin_bit_cast(v8bf, h);
                wlo[b] = __builtin_bit_cast(v8bf, l);
            } else {
#pragma unroll
                for (int s = 0; s < KSU; ++s) wop[b][s] = wsrc[(size_t)(4 * s + i4) * N + nvox[b]];
            }
#pragma unroll
            for (int rb = 0; rb < RBM; ++rb) yacc[b][rb] = V4{0, 0, 0, 0};
        }
        // the w operands arrive before the chunk loop starts. Without this wait the
        // compiler cannot count the loads still in flight inside the loop: it waits
        // for every one (the previous chunk's z stores too), or for the chunk
        // prefetch it has just issued, stalling each chunk on its own loads.
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)

        for (int c = 0; c < a.nchunk; ++c, ++g) {
            int cb = 0;                  // LDS buffer holding chunk c
            if constexpr (DBL) {
                // ---- the next chunk of the stream into the other buffer (free since
                //      the last barrier), then the loads of the one after it
                cb = g & 1;
                if (c + 1 < a.nchunk || more) stage(cb ^ 1);
                fetch();
            } else {
                // ---- chunk c: registers -> LDS; the loads of chunk c+1 stay in
                //      flight during the arithmetic of chunk c
                stage(0);
                __syncthreads();
                fetch();
            }
            // keep the loads ahead of the arithmetic (float64 has no registers to spare)
            if constexpr (MODE != MODE_FP64) __builtin_amdgcn_sched_barrier(0);

            const __amdgpu_buffer_rsrc_t zo = rsrc((T *)a.znew + (size_t)c * chunk_elems, chunk_bytes);

            // V operands of this chunk (one value per lane, see the host layout)
            T vu[BF ? 1 : KSU];
            T vy[BF ? 1 : RBM][4];
            T vt[TAIL ? 4 : 1][4];           // V[node 4 (l/16) + i][16 + t] for the tail ranks
            v8bf vuh, vul;
            v4s vyh[RB], vyl[RB];
            if constexpr (BF) {
                const v4u *U8 = (const v4u *)ldsv[cb];                      // [hi/lo][lane] x 8 bf16
                vuh = __builtin_bit_cast(v8bf, U8[lane]);
                vul = __builtin_bit_cast(v8bf, U8[64 + lane]);
                const v2u *Y4 = (const v2u *)((const char *)ldsv[cb] + 2048); // [rb][hi/lo][lane] x 4 bf16
    #pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    vyh[rb] = __builtin_bit_cast(v4s, Y4[(rb * 2 + 0) * 64 + lane]);
                    vyl[rb] = __builtin_bit_cast(v4s, Y4[(rb * 2 + 1) * 64 + lane]);
                }
            } else {
                const T *VT = (const T *)ldsv[cb];
    #pragma unroll
                for (int s = 0; s < KSU; ++s) vu[s] = VT[s * 64 + lane];
    #pragma unroll
                for (int rb = 0; rb < RBM; ++rb)
    #pragma unroll
                    for (int i = 0; i < 4; ++i) vy[rb][i] = VT[(KS + rb * 4 + i) * 64 + lane];
                if constexpr (TAIL) {
                    const T *VTt = VT + (KS + 4) * 64 + i4 * 16;   // tail table, see the host layout
    #pragma unroll
                    for (int i = 0; i < 4; ++i)
    #pragma unroll
                        for (int t = 0; t < 4; ++t) vt[i][t] = VTt[i * 4 + t];
                }
            }

            // when the rows of a wave stack along z, this lane's z^k of every row
            // is read once and also serves as the z neighbours of the adjacent rows
            const V4 *L = lds[cb] + i4 * B::NSP;
            // (float64 keeps the LDS stencil: built with x neighbours by DPP on both
            // 32-bit halves, the compiled code shifted only the first of the four
            // doubles and reused its neighbour sum for the other three)
            constexpr bool ZREG = TY == NW && MODE != MODE_FP64;   // row b + 1 of a wave is one step along z
            V4 zcs[ZREG ? BPW : 1];
            if constexpr (ZREG) {
    #pragma unroll
                for (int b = 0; b < BPW; ++b) zcs[b] = L[slot0[b]];
            }
    #pragma unroll
            for (int b = 0; b < BPW; ++b) {
                // u = V_r w^k for 16 nodes x 16 voxels
                V4 u = V4{0, 0, 0, 0};
                if constexpr (BF) {
                    // three split products, small terms first: lo*hi + hi*lo + hi*hi
                    u = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vul, whi[b], u, 0, 0, 0);
                    u = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vuh, wlo[b], u, 0, 0, 0);
                    u = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vuh, whi[b], u, 0, 0, 0);
                } else {
    #pragma unroll
                    for (int s = 0; s < KSU; ++s) u = F::mfma(vu[s], wop[b][s], u);
                }
                // D^T D z^k on the four planes of this lane: neighbours outside the grid
                // were staged as zeros, so deg * z - sum(neighbours) is exact
                const int sl = slot0[b];
                constexpr int SZ = B::SX * B::SY;
                V4 zc, nsum;
                if constexpr (ZREG) {
                    // x: the adjacent lanes of the row (DPP), the halo slot only at the
                    // row ends; y from LDS; z from this lane's other rows when adjacent
                    zc = zcs[ZREG ? b : 0];
                    V4 hm = V4{0, 0, 0, 0}, hp = V4{0, 0, 0, 0};
                    if (j == 0) hm = L[sl - 1];
                    if (j == 15) hp = L[sl + 1];
                    const V4 xm = dpp_x<true>(hm, zc), xp = dpp_x<false>(hp, zc);
                    const V4 zm = b > 0 ? zcs[b > 0 ? b - 1 : 0] : L[sl - SZ];
                    const V4 zp = b + 1 < BPW ? zcs[b + 1 < BPW ? b + 1 : 0] : L[sl + SZ];
                    nsum = (xm + xp) + (L[sl - B::SX] + L[sl + B::SX]) + (zm + zp);
                } else {
                    zc = L[sl];
                    nsum = (L[sl - 1] + L[sl + 1]) + (L[sl - B::SX] + L[sl + B::SX]) +
                           (L[sl - SZ] + L[sl + SZ]);
                }
                const V4 lap = deg[b] * zc - nsum;
                // projected z-update (Eq. z2 with f substituted)
                V4 zn = zc - tau * (lam2 * lap - beta * u);
    #pragma unroll
                for (int i = 0; i < 4; ++i) zn[i] = (zn[i] > (T)0 && inside[b]) ? zn[i] : (T)0;
                IO::store(zn, zo, soff[b]);
                if constexpr (MON) {
    #pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const T dd = zn[i] - zc[i];      // 0 outside the grid
                        dzacc += dd * dd;
                    }
                }
                if constexpr (BF) {
                    // K = the 16 nodes of the chunk in their natural lane order
                    v4s zh, zl;
                    split4(zn, zh, zl);
    #pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        yacc[b][rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(vyl[rb], zh, yacc[b][rb], 0, 0, 0);
                        yacc[b][rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(vyh[rb], zl, yacc[b][rb], 0, 0, 0);
                        yacc[b][rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(vyh[rb], zh, yacc[b][rb], 0, 0, 0);
                    }
                } else {
                    // y^{k+1} += V_r^T z^{k+1}: K-row l/16 of step i is node 4*(l/16)+i
    #pragma unroll
                    for (int rb = 0; rb < RBM; ++rb)
    #pragma unroll
                        for (int i = 0; i < 4; ++i)
                            yacc[b][rb] = F::mfma(vy[rb][i], zn[i], yacc[b][rb]);
                    if constexpr (TAIL) {
    #pragma unroll
                        for (int t = 0; t < 4; ++t)
    #pragma unroll
                            for (int i = 0; i < 4; ++i) ytail[b][t] += vt[i][t] * zn[i];
                    }
                }
            }
            __syncthreads();
        }

        // ---- tail ranks: sum the four node groups (lanes j, j+16, j+32, j+48)
        if constexpr (TAIL) {
    #pragma unroll
            for (int b = 0; b < BPW; ++b)
    #pragma unroll
                for (int t = 0; t < 4; ++t) {
                    T v = ytail[b][t];
                    v += __shfl_xor(v, 16);
                    v += __shfl_xor(v, 32);
                    ytail[b][t] = v;
                }
        }

        // ---- r-vector recursion (lane holds y^{k+1}[r][voxel j] for the four ranks r
        //      of its accumulator rows). The double-buffered bricks issue a row's
        //      loads before forming any result (measured 1 % faster for float32; the
        //      other shapes measured slower with it and keep one rank at a time).
        if constexpr (DBL) {
            // padded ranks and voxels outside the grid get out-of-range offsets: their
            // loads return 0 and their stores are dropped
            const unsigned rbytes = (unsigned)((size_t)a.RP * N * sizeof(T));
            const __amdgpu_buffer_rsrc_t wr = rsrc(a.w, rbytes), yr = rsrc(a.y, rbytes), ahr = rsrc(a.ah, rbytes),
                                         bcr = rsrc(a.bcoef, (unsigned)(a.RP * sizeof(T)));
            auto ld1 = [](const __amdgpu_buffer_rsrc_t &rs, unsigned off) -> T {
                if constexpr (sizeof(T) == 8)
                    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
                else
                    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
            };
        #pragma unroll
            for (int b = 0; b < BPW; ++b) {
                T lah[RB][4], lyo[RB][4], lw[RB][4], lbc[RB][4];
                unsigned ob[RB][4];
        #pragma unroll
                for (int rb = 0; rb < RB; ++rb)
        #pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        // f64 16x16x4 returns rows l/16 + 4 i; the others rows 4 (l/16) + i
                        const int r = MODE == MODE_FP64 ? 16 * rb + i4 + 4 * i : 16 * rb + 4 * i4 + i;
                        const size_t o = (size_t)r * N + nvox[b];
                        ob[rb][i] = r < a.r && valid[b] ? (unsigned)(o * sizeof(T)) : OOB;
                        const unsigned obc = r < a.r ? (unsigned)(r * sizeof(T)) : OOB;
                        lah[rb][i] = ld1(ahr, ob[rb][i]);
                        lyo[rb][i] = ld1(yr, ob[rb][i]);
                        lw[rb][i] = ld1(wr, ob[rb][i]);
                        lbc[rb][i] = ld1(bcr, obc);
                    }
        #pragma unroll
                for (int rb = 0; rb < RB; ++rb)
        #pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int r = MODE == MODE_FP64 ? 16 * rb + i4 + 4 * i : 16 * rb + 4 * i4 + i;
                        T yn;
                        if constexpr (TAIL) {
                            if (rb == 0) {
                                yn = yacc[b][0][i];
                            } else {                     // r in 16..19 here (a.r <= 20)
                                const int t = r - 16;
                                yn = t == 0 ? ytail[b][0] : t == 1 ? ytail[b][1] : t == 2 ? ytail[b][2] : ytail[b][3];
                            }
                        } else {
                            yn = yacc[b][rb][i];
                        }
                        const T wn = lah[rb][i] - lbc[rb][i] * ((T)2 * yn - lyo[rb][i] - lw[rb][i]);
                        if constexpr (sizeof(T) == 8) {
                            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, wn), wr, ob[rb][i], 0, 0);
                            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, yn), yr, ob[rb][i], 0, 0);
                        } else {
                            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, wn), wr, ob[rb][i], 0, 0);
                            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, yn), yr, ob[rb][i], 0, 0);
                        }
                    }
            }
        } else {
            const T *ah = (const T *)a.ah;
            const T *bc = (const T *)a.bcoef;
            const unsigned rbytes = (unsigned)((size_t)a.RP * N * sizeof(T));
            const __amdgpu_buffer_rsrc_t wr = rsrc(a.w, rbytes), yr = rsrc(a.y, rbytes);
            const T *yold = (const T *)a.y;
        #pragma unroll
            for (int b = 0; b < BPW; ++b) {
        #pragma unroll
                for (int rb = 0; rb < RB; ++rb)
        #pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        // f64 16x16x4 returns rows l/16 + 4 i; the others rows 4 (l/16) + i
                        const int r = MODE == MODE_FP64 ? 16 * rb + i4 + 4 * i : 16 * rb + 4 * i4 + i;
                        if (r >= a.r) continue;          // padded ranks stay 0 (never stored)
                        const size_t o = (size_t)r * N + nvox[b];
                        T yn;
                        if constexpr (TAIL) {
                            if (rb == 0) {
                                yn = yacc[b][0][i];
                            } else {                     // r in 16..19 here (a.r <= 20)
                                const int t = r - 16;
                                yn = t == 0 ? ytail[b][0] : t == 1 ? ytail[b][1] : t == 2 ? ytail[b][2] : ytail[b][3];
                            }
                        } else {
                            yn = yacc[b][rb][i];
                        }
                        const T wn = ah[o] - bc[r] * ((T)2 * yn - yold[o] - wsrc[o]);
                        const unsigned ob = valid[b] ? (unsigned)(o * sizeof(T)) : OOB;
                        if constexpr (sizeof(T) == 8) {
                            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, wn), wr, ob, 0, 0);
                            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, yn), yr, ob, 0, 0);
                        } else {
                            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, wn), wr, ob, 0, 0);
                            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, yn), yr, ob, 0, 0);
                        }
                    }
            }
        }
        if constexpr (MON) {
            brick_sum_out<NW>((double)dzacc, mred, mon, tile);
            dzacc = 0;
        }
        if constexpr (!DBL) break;   // one brick per workgroup
    }
}

// ---------------------------------------------------------------------------
// Variant with the chunk staged by direct buffer->LDS loads (used for bf16x3;
// it also compiles for float32).
//
// The brick's halo box (SX x SY x SZ voxel slots, 64 B each) is copied into
// LDS by buffer_load ... lds, which writes lane k's 16 bytes to entry k of a
// 1 KB run; no registers hold the data in flight. Two LDS buffers alternate:
// chunk c+1 lands in one while chunk c is read from the other, so a single
// barrier per chunk suffices. Inside a slot the four 16-byte quads are
// XOR-swizzled by bits 2..3 of the slot index, so the sixteen lanes of a row
// (sixteen consecutive slots, one quad) hit sixteen distinct bank groups.
// z^{k+1} of chunk c is written at the start of chunk c+1 (deferred), so the
// wait for chunk c+1's loads never stalls on stores just issued.
template <int TY, int TZ> struct Box {
    static constexpr int SX = TX + 2, SY = TY + 2, SZ = TZ + 2;
    static constexpr int NS = SX * SY * SZ;       // slots
    static constexpr int NE = NS * 4;             // 16-byte entries
    static constexpr int NG = (NE + 63) / 64;     // 64-entry load groups
};

__device__ __forceinline__ int swz(int slot) { return (slot >> 2) & 3; }

// 16 bytes per lane from a buffer straight into LDS: lane k fills the k-th
// 16-byte entry after `lds` (wave-uniform base).
__device__ __forceinline__ void lds_dma16(__amdgpu_buffer_rsrc_t r, void *lds, unsigned voff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void *)lds, 16,
                                             voff, 0, 0, 0);
}

template <int MODE, int RB, int KSU, int TY, int TZ, bool MON>
__global__ void __launch_bounds__(NT, 1)
k_fused_dma(const IterArgs *__restrict__ jobs, const TileRef *__restrict__ tiles, int ntiles,
        int round, double *__restrict__ mon) {
    static_assert(MODE != MODE_FP64, "float64 uses the register-staged kernel");
    using F = FT<MODE>;
    using V4 = v4f;
    using BX = Box<TY, TZ>;
    constexpr bool BF = MODE == MODE_BF16X3;
    constexpr int NW = NT / 64;
    constexpr int NB = TY * TZ;
    constexpr int BPW = NB / NW;
    constexpr int GPW = (BX::NG + NW - 1) / NW;   // load groups per wave
    constexpr int VB = VopSize<MODE, RB>::bytes;
    constexpr int VG = VB / 1024;                 // V load groups (waves 0 .. VG-1)
    constexpr int KS = 4 * RB;
    static_assert(NB % NW == 0, "brick rows must split over the waves");
    static_assert(VB % 1024 == 0 && VG <= NW, "V block must be whole load groups");
    static_assert(BF || (KSU >= 1 && KSU <= KS), "u K-steps must fit the padded rank");

    __shared__ uint4 zbuf[2][BX::NG * 64];
    __shared__ uint4 vbuf[2][VB / 16];
    __shared__ double mred[MON ? NW : 1];
    float dzacc = 0.0f;

    int tile = blockIdx.x;
    if ((ntiles & 7) == 0) {             // keep neighbouring bricks on one XCD (shared L2)
        const int per = ntiles >> 3;
        tile = (tile & 7) * per + (tile >> 3);
    }
    const TileRef tr = tiles[tile];
    // two descriptors per job (z^k -> z^{k+1} for even and odd k); a job that
    // joined a shared loop late carries its phase
    const int sel = (round + jobs[2 * tr.job].phase) & 1;
    const IterArgs &a = jobs[2 * tr.job + sel];
    const int64_t nx = a.g.nx, ny = a.g.ny, nz = a.g.nz, N = a.g.N;
    const int64_t x0 = (int64_t)tr.tx * TX, y0 = (int64_t)tr.ty * TY, z0 = (int64_t)tr.tz * TZ;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int j = lane & 15;
    const int i4 = lane >> 4;

    const float tau = (float)a.tau, lam2 = (float)a.lam2, beta = (float)a.beta;
    const size_t chunk_elems = (size_t)N * QC;
    const unsigned chunk_bytes = (unsigned)(chunk_elems * sizeof(float));

    // ---- load descriptors: entry e = 64 g + lane of the box -> slot e/4, stored
    //      position e%4 holds quad (e%4) ^ swz(slot) of that voxel's chunk
    unsigned voff[GPW];
#pragma unroll
    for (int i = 0; i < GPW; ++i) {
        const int e = 64 * (wave + NW * i) + lane;
        const int sl = e >> 2;
        voff[i] = OOB;
        if (sl < BX::NS) {
            const int q = (e & 3) ^ swz(sl);
            const int sx = sl % BX::SX, sy = (sl / BX::SX) % BX::SY, sz = sl / (BX::SX * BX::SY);
            const int64_t gx = x0 + sx - 1, gy = y0 + sy - 1, gz = z0 + sz - 1;
            // edge and corner slots of the halo box are never read: leave them unloaded
            const int rim = (sx == 0 || sx == BX::SX - 1) + (sy == 0 || sy == BX::SY - 1) +
                            (sz == 0 || sz == BX::SZ - 1);
            if (rim < 2 && gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz)
                voff[i] = (unsigned)(((gx + nx * (gy + ny * gz)) * QC + 4 * q) * sizeof(float));
        }
    }
    const __amdgpu_buffer_rsrc_t vrs = rsrc(a.Vu, (unsigned)(a.nchunk * VB));
    auto issue = [&](int c) {
        const int b = c & 1;
        const __amdgpu_buffer_rsrc_t zr = rsrc((const float *)a.z + (size_t)c * chunk_elems, chunk_bytes);
#pragma unroll
        for (int i = 0; i < GPW; ++i) {
            const int g = wave + NW * i;
            if (g < BX::NG) lds_dma16(zr, &zbuf[b][64 * g], voff[i]);
        }
        if (wave < VG)
            lds_dma16(vrs, &vbuf[b][64 * wave], (unsigned)(c * VB + 1024 * wave + 16 * lane));
    };

    // ---- per-row voxel coordinates and LDS byte addresses of the 7-point stencil
    int64_t nvox[BPW];
    bool valid[BPW];
    float deg[BPW];
    bool inside[BPW];                    // false: outside a mask (z stays 0)
    unsigned soff[BPW];
    int sa[BPW][7];                      // byte offsets inside a z buffer
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
        const int row = wave + NW * b;
        const int by = row % TY, bz = row / TY;
        const int64_t gx = x0 + j, gy = y0 + by, gz = z0 + bz;
        valid[b] = gx < nx && gy < ny && gz < nz;
        nvox[b] = valid[b] ? gx + nx * (gy + ny * gz) : 0;
        deg[b] = (float)((gx > 0) + (gx + 1 < nx) + (gy > 0) + (gy + 1 < ny) + (gz > 0) + (gz + 1 < nz));
        inside[b] = valid[b];            // lanes beyond the grid compute z^{k+1} = 0 (never stored)
        if (a.code) {
            const unsigned cb = a.code[nvox[b]];
            deg[b] = (float)(cb & 7u);
            inside[b] = valid[b] && (cb & 0x80u) != 0;
        }
        soff[b] = valid[b] ? (unsigned)((nvox[b] * QC + 4 * i4) * sizeof(float)) : OOB;
        const int s0 = (j + 1) + BX::SX * ((by + 1) + BX::SY * (bz + 1));
        const int nb[7] = {s0, s0 - 1, s0 + 1, s0 - BX::SX, s0 + BX::SX, s0 - BX::SX * BX::SY,
                           s0 + BX::SX * BX::SY};
#pragma unroll
        for (int k = 0; k < 7; ++k) sa[b][k] = 64 * nb[k] + 16 * (i4 ^ swz(nb[k]));
    }

    // ---- u operand (see k_fused)
    const float *wsrc = (const float *)a.w;
    float wop[BPW][BF ? 1 : KSU];
    v8bf whi[BF ? BPW : 1], wlo[BF ? BPW : 1];
    V4 yacc[BPW][RB];
    V4 zkeep[BPW];
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
        if constexpr (BF) {
            v4u h = v4u{0, 0, 0, 0}, l = v4u{0, 0, 0, 0};
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) {
                const int r = 8 * i4 + jj;
                const float v = r < a.RP ? wsrc[(size_t)r * N + nvox[b]] : 0.0f;
                const unsigned hb = bf16_bits(v);
                const unsigned lb = bf16_bits(v - bf16_val(hb));
                h[jj >> 1] |= hb << (16 * (jj & 1));
                l[jj >> 1] |= lb << (16 * (jj & 1));
            }
            whi[b] = __builtin_bit_cast(v8bf, h);
            wlo[b] = __builtin_bit_cast(v8bf, l);
        } else {
#pragma unroll
            for (int s = 0; s < KSU; ++s) wop[b][s] = wsrc[(size_t)(4 * s + i4) * N + nvox[b]];
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) yacc[b][rb] = V4{0, 0, 0, 0};
        zkeep[b] = V4{0, 0, 0, 0};
    }

    issue(0);
    for (int c = 0; c < a.nchunk; ++c) {
        // this wave's loads of chunk c (and its stores of chunk c-1) are done;
        // the barrier makes every wave's part visible and frees the other buffer
        __builtin_amdgcn_s_waitcnt(0x0F70);          // vmcnt(0)
        __syncthreads();
        if (c > 0) {                                  // deferred z^{k+1} of chunk c-1
            const __amdgpu_buffer_rsrc_t zo =
                rsrc((float *)a.znew + (size_t)(c - 1) * chunk_elems, chunk_bytes);
#pragma unroll
            for (int b = 0; b < BPW; ++b) Buf<float, v4f>::store(zkeep[b], zo, soff[b]);
        }
        if (c + 1 < a.nchunk) issue(c + 1);
        const int bsel = c & 1;
        const char *Z = (const char *)&zbuf[bsel][0];

        float vu[BF ? 1 : KSU];
        float vy[BF ? 1 : RB][4];
        v8bf vuh, vul;
        v4s vyh[RB], vyl[RB];
        if constexpr (BF) {
            const v4u *U8 = (const v4u *)&vbuf[bsel][0];
            vuh = __builtin_bit_cast(v8bf, U8[lane]);
            vul = __builtin_bit_cast(v8bf, U8[64 + lane]);
            const v2u *Y4 = (const v2u *)((const char *)&vbuf[bsel][0] + 2048);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                vyh[rb] = __builtin_bit_cast(v4s, Y4[(rb * 2 + 0) * 64 + lane]);
                vyl[rb] = __builtin_bit_cast(v4s, Y4[(rb * 2 + 1) * 64 + lane]);
            }
        } else {
            const float *VT = (const float *)&vbuf[bsel][0];
#pragma unroll
            for (int s = 0; s < KSU; ++s) vu[s] = VT[s * 64 + lane];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) vy[rb][i] = VT[(KS + rb * 4 + i) * 64 + lane];
        }

#pragma unroll
        for (int b = 0; b < BPW; ++b) {
            V4 u = V4{0, 0, 0, 0};
            if constexpr (BF) {
                u = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vul, whi[b], u, 0, 0, 0);
                u = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vuh, wlo[b], u, 0, 0, 0);
                u = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vuh, whi[b], u, 0, 0, 0);
            } else {
#pragma unroll
                for (int s = 0; s < KSU; ++s) u = F::mfma(vu[s], wop[b][s], u);
            }
            const V4 zc = *(const V4 *)(Z + sa[b][0]);
            const V4 nsum = (*(const V4 *)(Z + sa[b][1]) + *(const V4 *)(Z + sa[b][2])) +
                            (*(const V4 *)(Z + sa[b][3]) + *(const V4 *)(Z + sa[b][4])) +
                            (*(const V4 *)(Z + sa[b][5]) + *(const V4 *)(Z + sa[b][6]));
            const V4 lap = deg[b] * zc - nsum;
            V4 zn = zc - tau * (lam2 * lap - beta * u);
#pragma unroll
            for (int i = 0; i < 4; ++i) zn[i] = (zn[i] > 0.0f && inside[b]) ? zn[i] : 0.0f;
            zkeep[b] = zn;
            if constexpr (MON) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float dd = zn[i] - zc[i];      // 0 outside the grid
                    dzacc += dd * dd;
                }
            }
            if constexpr (BF) {
                v4s zh, zl;
                split4(zn, zh, zl);
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    yacc[b][rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(vyl[rb], zh, yacc[b][rb], 0, 0, 0);
                    yacc[b][rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(vyh[rb], zl, yacc[b][rb], 0, 0, 0);
                    yacc[b][rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(vyh[rb], zh, yacc[b][rb], 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        yacc[b][rb] = F::mfma(vy[rb][i], zn[i], yacc[b][rb]);
            }
        }
    }
    {
        const __amdgpu_buffer_rsrc_t zo =
            rsrc((float *)a.znew + (size_t)(a.nchunk - 1) * chunk_elems, chunk_bytes);
#pragma unroll
        for (int b = 0; b < BPW; ++b) Buf<float, v4f>::store(zkeep[b], zo, soff[b]);
    }

    // ---- r-vector recursion: gather, then update, then store
    const float *ah = (const float *)a.ah;
    const float *bc = (const float *)a.bcoef;
    const unsigned rbytes = (unsigned)((size_t)a.RP * N * sizeof(float));
    const __amdgpu_buffer_rsrc_t wr = rsrc(a.w, rbytes), yr = rsrc(a.y, rbytes);
    const float *yold = (const float *)a.y;
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
        float ahv[RB][4], yov[RB][4], wov[RB][4], bcv[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * rb + 4 * i4 + i;
                const size_t o = (size_t)r * N + nvox[b];
                ahv[rb][i] = ah[o];
                yov[rb][i] = yold[o];
                wov[rb][i] = wsrc[o];
                bcv[rb][i] = bc[r];
            }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * rb + 4 * i4 + i;
                const unsigned ob = valid[b] ? (unsigned)(((size_t)r * N + nvox[b]) * sizeof(float)) : OOB;
                const float yn = yacc[b][rb][i];
                const float wn = ahv[rb][i] - bcv[rb][i] * (2.0f * yn - yov[rb][i] - wov[rb][i]);
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, wn), wr, ob, 0, 0);
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, yn), yr, ob, 0, 0);
            }
    }
    if constexpr (MON) brick_sum_out<NW>((double)dzacc, mred, mon, tile);
}

// Longest brick (in 16-node chunks) that the double-buffered shapes run persistent.
constexpr int kPersistChunks = 32;

// Compute units of the current device (the persistent grid's width), read once per device.
int device_cus() {
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

template <int MODE, int RB, int KSU, int TY, int TZ, bool MON>
void launch_t(const FusedLaunch &L, hipStream_t s) {
    // bf16x3 stages the small volumetric brick through registers (four waves
    // per SIMD) and the others through direct LDS loads; float32 and float64
    // always through registers
    if constexpr (MODE == MODE_BF16X3 && !fused_small(MODE, TY, TZ))
        hipLaunchKernelGGL((k_fused_dma<MODE, RB, KSU, TY, TZ, MON>), dim3(L.ntiles), dim3(NT), 0, s,
                           L.jobs, L.tiles, L.ntiles, L.round, L.mon);
    else {
        // Short bricks of the double-buffered shapes (one workgroup per CU) run a
        // persistent grid, at most one workgroup per CU: the loads of a brick's
        // first chunks then overlap the end of the brick before. Measured per
        // iteration: float32 128 x 128 x 64 at 9 chunks 3 % faster, equal at
        // 25..49; float64 512 x 512 at 7 chunks 5 % faster; float32 512 x 512 at
        // 25 chunks 4 % faster. Long bricks take one workgroup each: the
        // hardware's dynamic dispatch balances them better than a fixed share per
        // CU (float32 volumetric at 100 chunks: 1 % slower persistent).
        int nwg = L.ntiles;
        if constexpr ((MODE == MODE_FP32 && ((TY == 8 && TZ == 4) || (TY == 16 && TZ == 1))) ||
                      (MODE == MODE_FP64 && ((TY == 8 && TZ == 1) || (TY == 4 && TZ == 2)))) {
            const int cus = device_cus();
            if (L.maxchunk > 0 && L.maxchunk <= kPersistChunks && cus > 0 && cus < nwg) nwg = cus;
        }
        hipLaunchKernelGGL((k_fused<MODE, RB, KSU, TY, TZ, MON>), dim3(nwg), dim3(NT), 0, s, L.jobs,
                           L.tiles, L.ntiles, L.round, L.mon);
    }
}

// Monitored iterations (L.mon set) run the variant that also sums (z^{k+1} - z^k)^2.
template <int MODE, int RB, int KSU, int TY, int TZ>
void launch_m(const FusedLaunch &L, hipStream_t s) {
    if (L.mon) launch_t<MODE, RB, KSU, TY, TZ, true>(L, s);
    else launch_t<MODE, RB, KSU, TY, TZ, false>(L, s);
}

template <int MODE, int RB, int KSU>
bool launch_shape(const FusedLaunch &L, hipStream_t s) {
    const int ty = L.shape.ty, tz = L.shape.tz;
    if constexpr (MODE == MODE_FP64) {
        if (ty == 8 && tz == 1) return launch_m<MODE, RB, KSU, 8, 1>(L, s), true;
        if (ty == 16 && tz == 1) return launch_m<MODE, RB, KSU, 16, 1>(L, s), true;
        if (ty == 4 && tz == 4) return launch_m<MODE, RB, KSU, 4, 4>(L, s), true;
        if (ty == 4 && tz == 2) return launch_m<MODE, RB, KSU, 4, 2>(L, s), true;
    } else {
        if (ty == 8 && tz == 1) return launch_m<MODE, RB, KSU, 8, 1>(L, s), true;
        if (ty == 16 && tz == 1) return launch_m<MODE, RB, KSU, 16, 1>(L, s), true;
        if (ty == 4 && tz == 4) return launch_m<MODE, RB, KSU, 4, 4>(L, s), true;
        if (ty == 8 && tz == 4) return launch_m<MODE, RB, KSU, 8, 4>(L, s), true;
        if constexpr (MODE == MODE_BF16X3)
            if (ty == 4 && tz == 2) return launch_m<MODE, RB, KSU, 4, 2>(L, s), true;
        if constexpr (MODE == MODE_FP32)
            if (ty == 32 && tz == 1) return launch_m<MODE, RB, KSU, 32, 1>(L, s), true;
    }
    return false;
}

// u K-steps: r <= 16 -> 4, 17..20 -> 5, 21..24 -> 6, 25..32 -> 8 (zero-padded ranks)
template <int MODE>
bool launch_mode(const FusedLaunch &L, hipStream_t s) {
    if (L.r <= 16) return launch_shape<MODE, 1, 4>(L, s);
    if (L.r <= 20) return launch_shape<MODE, 2, 5>(L, s);
    if (L.r <= 24) return launch_shape<MODE, 2, 6>(L, s);
    return launch_shape<MODE, 2, 8>(L, s);
}

}  // namespace

bool fused_supported(int mode, int RP, int64_t N) {
    // buffer offsets are 32-bit and must stay below the out-of-range marker
    const int64_t esz = mode == MODE_FP64 ? 8 : 4;
    return (mode == MODE_FP32 || mode == MODE_FP64 || mode == MODE_BF16X3) &&
           (RP == 16 || RP == 32) && N * QC * esz < ((int64_t)1 << 31) &&
           (int64_t)RP * N * esz < ((int64_t)1 << 31);
}

FusedShape default_shape(int mode, const Grid &g) {
    // Bricks per grid for a shape; a grid whose bricks would not fill the CUs is
    // latency-bound, and a thinner brick (more workgroups) pays there.
    const int dc = device_cus();
    const int cus = dc > 0 ? dc : 256;
    auto bricks = [&](int ty, int tz) -> int64_t {
        return ((g.nx + 15) / 16) * ((g.ny + ty - 1) / ty) * ((g.nz + tz - 1) / tz);
    };
    // float64 planar: the double-buffered 16 x 8 x 1 brick (32 x 32 with Q = 100:
    // 31.3 -> 18.3 us per iteration against 16 x 16 x 1; 1024 x 1024: 777 -> 745 us).
    // float64 volumetric: 16 x 4 x 4, or the double-buffered 16 x 4 x 2 when the
    // 16 x 4 x 4 bricks would not fill the CUs (32 x 32 x 32 with Q = 100: 34.0 ->
    // 23.8 us; from 64 x 64 x 32 up 16 x 4 x 4 is 7-17 % faster)
    if (mode == MODE_FP64) {
        if (g.nz == 1) return FusedShape{8, 1};
        return bricks(4, 4) < cus ? FusedShape{4, 2} : FusedShape{4, 4};
    }
    // bf16x3 planar: the 16 x 8 x 1 direct-LDS brick (two workgroups per CU) beat
    // 16 x 16 x 1 at every size measured (128 x 128: 144 -> 106 us per iteration,
    // 1024 x 1024: 956 -> 850 us). bf16x3 volumetric: 16 x 4 x 4, or 16 x 4 x 2 when
    // the 16 x 4 x 4 bricks would not fill the CUs (32 x 32 x 32: 94.7 -> 75.0 us;
    // at 288 bricks equal, at 384 16 x 4 x 4 is 9 % faster)
    if (mode == MODE_BF16X3) {
        if (g.nz == 1) return FusedShape{8, 1};
        return bricks(4, 4) < cus ? FusedShape{4, 2} : FusedShape{4, 4};
    }
    // float32 planar: the double-buffered 16 x 16 x 1 brick, or 16 x 8 x 1 (several
    // workgroups per CU) while its bricks fit one per CU (128 x 128 with Q = 1600:
    // 160 -> 121 us per iteration; 176 x 176: 168 -> 131 us; 200 x 180, 299 such
    // bricks: 174 against 186 us, so 16 x 16 x 1 there).
    // float32 volumetric: 16 x 8 x 4, or 16 x 4 x 4 (twice the bricks, two
    // workgroups per CU) when the 16 x 8 x 4 bricks would not fill the CUs
    // (32 x 32 x 32 with Q = 400: 86.6 -> 51.6 us per iteration; 48 x 48 x 32 with
    // Q = 1600: 332 -> 310 us)
    if (g.nz == 1) return bricks(8, 1) < cus ? FusedShape{8, 1} : FusedShape{16, 1};
    return bricks(8, 4) < cus ? FusedShape{4, 4} : FusedShape{8, 4};
}

std::vector<FusedShape> candidate_shapes(int mode, bool planar) {
    if (mode == MODE_FP64) return planar ? std::vector<FusedShape>{{8, 1}, {16, 1}} : std::vector<FusedShape>{{4, 4}, {4, 2}};
    if (planar) {
        if (mode == MODE_FP32) return {{8, 1}, {16, 1}, {32, 1}};
        return {{8, 1}, {16, 1}};
    }
    if (mode == MODE_BF16X3) return {{4, 4}, {4, 2}, {8, 4}};
    return {{4, 4}, {8, 4}};
}

void append_tiles(const Grid &g, int job, int mode, FusedShape sh, std::vector<TileRef> &out,
                  const std::vector<uint8_t> *code) {
    const int tx = (int)((g.nx + 15) / 16), ty = (int)((g.ny + sh.ty - 1) / sh.ty),
              tz = (int)((g.nz + sh.tz - 1) / sh.tz);
    // Bricks that run at the same time on one XCD can share their face halos
    // through its L2. The float32 16 x 8 x 4 brick (one workgroup per CU, 32 per
    // XCD) lists its bricks in blocks of 8 x 2 x 2 (x fastest inside a block, then
    // y, then z; the blocks in x, y, z order). At 128 x 128 x 64 (8 x 16 x 16
    // bricks) this measured about 1 % faster than blocks of 4 x 8 x 1 and 3.5 %
    // faster than x-fastest rows; blocks two bricks wide (2 x 4 x 4, 2 x 2 x 8)
    // read fewer bytes but ran 8 % slower. The 16 x 4 x 4 bricks ran 8-12 %
    // slower with any blocking tried (2 x 8 x 4, 3 x 4 x 4, 6 x 4 x 2, ...), so
    // every other shape keeps the plain order.
    const bool blocked = mode == MODE_FP32 && sh.ty == 8 && sh.tz == 4;
    const int bx = blocked ? 8 : tx, by = blocked ? 2 : ty, bz = blocked ? 2 : 1;
    for (int k0 = 0; k0 < tz; k0 += bz)
        for (int j0 = 0; j0 < ty; j0 += by)
            for (int i0 = 0; i0 < tx; i0 += bx)
                for (int k = k0; k < std::min(k0 + bz, tz); ++k)
                    for (int jy = j0; jy < std::min(j0 + by, ty); ++jy)
                        for (int i = i0; i < std::min(i0 + bx, tx); ++i)
                            if (!code || brick_has_inside(g, *code, (int64_t)i * TX, (int64_t)jy * sh.ty,
                                                          (int64_t)k * sh.tz, TX, sh.ty, sh.tz))
                                out.push_back(TileRef{job, i, jy, k});
}

bool launch_fused(const FusedLaunch &L, hipStream_t s) {
    if (L.ntiles <= 0) return true;
    if (L.mode == MODE_FP64) return launch_mode<MODE_FP64>(L, s);
    if (L.mode == MODE_FP32) return launch_mode<MODE_FP32>(L, s);
    if (L.RP == 16) return launch_shape<MODE_BF16X3, 1, 1>(L, s);
    return launch_shape<MODE_BF16X3, 2, 1>(L, s);
}

namespace {
uint16_t host_bf16_bits(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
float host_bf16_val(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}
}  // namespace

// bf16 hi/lo operand images of the float32-rounded V for the split-precision
// fused kernel, one contiguous block per chunk c:
//   u part: [h][l][jj] = V[16 c + l % 16][8 (l / 16) + jj]        (A of u, K = rank, 32 wide)
//   y part: [rb][h][l][jj] = V[16 c + 4 (l / 16) + jj][16 rb + l % 16]  (A of y, K = 16 nodes)
// h = 0 holds the rounded value, h = 1 the rounded remainder.
void fused_operands_bf16(const std::vector<double> &Vh, int Qp, int RP, std::vector<uint16_t> &Vop) {
    const int nchunk = Qp / QC, RB = RP / 16;
    const size_t per = 2 * 64 * 8 + (size_t)RB * 2 * 64 * 4;   // uint16 per chunk
    Vop.assign((size_t)nchunk * per, 0);
    auto split = [](double v, uint16_t &h, uint16_t &l) {
        const float f = (float)v;
        h = host_bf16_bits(f);
        l = host_bf16_bits(f - host_bf16_val(h));
    };
    for (int c = 0; c < nchunk; ++c) {
        uint16_t *U = &Vop[(size_t)c * per];
        uint16_t *Y = U + 2 * 64 * 8;
        for (int l = 0; l < 64; ++l) {
            for (int jj = 0; jj < 8; ++jj) {
                const int r = 8 * (l / 16) + jj;
                const double v = r < RP ? Vh[(size_t)(16 * c + l % 16) * RP + r] : 0.0;
                uint16_t h, lo;
                split(v, h, lo);
                U[(0 * 64 + l) * 8 + jj] = h;
                U[(1 * 64 + l) * 8 + jj] = lo;
            }
            for (int rb = 0; rb < RB; ++rb)
                for (int jj = 0; jj < 4; ++jj) {
                    const double v = Vh[(size_t)(16 * c + 4 * (l / 16) + jj) * RP + 16 * rb + l % 16];
                    uint16_t h, lo;
                    split(v, h, lo);
                    Y[((rb * 2 + 0) * 64 + l) * 4 + jj] = h;
                    Y[((rb * 2 + 1) * 64 + l) * 4 + jj] = lo;
                }
        }
    }
}

// Operand images of V for the fused kernel (see the lane mapping above), one
// contiguous block of (KS + 4 RB) * 64 values per chunk c:
//   u part: [s][l]    = V[16 c + row(l % 16)][4 s + l / 16]       (A of u = V w)
//   y part: [rb][i][l] = V[16 c + 4 (l / 16) + i][16 rb + l % 16]  (A of y = V^T z)
// The f32 16x16x4 MFMA returns output rows 4 (l/16) + i in lane l, the f64
// one rows l/16 + 4 i; row() maps an MFMA output row of u to the chunk node
// that lane must hold (node 4 (l/16) + i): identity for f32, m -> 4 (m % 4)
// + m / 4 for f64.
void fused_operands(const std::vector<double> &Vh, int Qp, int RP, bool f64_rows, bool tail,
                    std::vector<double> &Vop) {
    const int nchunk = Qp / QC, RB = RP / 16, KS = 4 * RB;
    const size_t per = (size_t)(KS + 4 * RB) * 64;
    Vop.assign((size_t)nchunk * per, 0.0);
    for (int c = 0; c < nchunk; ++c) {
        double *U = &Vop[(size_t)c * per];
        double *Y = U + (size_t)KS * 64;
        for (int l = 0; l < 64; ++l) {
            const int m = l % 16;
            const int row = f64_rows ? 4 * (m % 4) + m / 4 : m;
            for (int s = 0; s < KS; ++s)
                U[s * 64 + l] = Vh[(size_t)(16 * c + row) * RP + 4 * s + l / 16];
            for (int rb = 0; rb < (tail ? 1 : RB); ++rb)
                for (int i = 0; i < 4; ++i)
                    Y[(rb * 4 + i) * 64 + l] =
                        Vh[(size_t)(16 * c + 4 * (l / 16) + i) * RP + 16 * rb + l % 16];
        }
        if (tail)   // [g][i][t] = V[node 4 g + i][rank 16 + t], g = lane / 16
            for (int g = 0; g < 4; ++g)
                for (int i = 0; i < 4; ++i)
                    for (int t = 0; t < 4; ++t)
                        Y[4 * 64 + (g * 4 + i) * 4 + t] = Vh[(size_t)(16 * c + 4 * g + i) * RP + 16 + t];
    }
}

}  // namespace ssmap
