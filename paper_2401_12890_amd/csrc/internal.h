// Internal interfaces of libssmap (not part of the C ABI).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <vector>

namespace ssmap {

// Iteration arithmetic (mirrors ssmap_precision).
enum Mode { MODE_FP64 = 0, MODE_FP32 = 1, MODE_BF16X3 = 2 };

// Spectral nodes are stored in chunks of QC consecutive q per voxel:
// element (q, n) lives at ((q / QC) * N + n) * QC + q % QC. Q is padded to a
// multiple of QC with rows of V equal to zero, which keeps padded z at 0.
constexpr int QC = 16;

// Monitoring reduction slots (float64 sums): data term ||m - K_r z||^2, forward-edge
// regulariser sum ||z_n - z_m||^2, ||z||^2, ||z - zprev||^2, non-finite count,
// ||z - f*||^2, ||f*||^2, ||z - f||^2, ||f - f*||^2.
enum { ST_DATA = 0, ST_REG, ST_ZNORM, ST_DZ, ST_NONFINITE, ST_DFCS, ST_FSTAR, ST_PRIMAL,
       ST_DFCS_F, ST_COUNT = 12 };

void thin_svd(const double *K, int P, int Q, std::vector<double> &U,
              std::vector<double> &s, std::vector<double> &V);

struct Grid {
    int64_t nx, ny, nz, N;
};

// Device pointers and scalars of one LADMM iteration in the reduced form
// (state z, plus per-voxel r-vectors w, y and the constant a*h).
struct IterArgs {
    const void *z;        // z^k      (chunked layout, Qp x N)
    void *znew;           // z^{k+1}
    void *w;              // w^k -> w^{k+1}   (RP x N, row i at i*N)
    void *y;              // y^k -> y^{k+1}   (RP x N)
    const void *ah;       // a .* h          (RP x N)
    const void *V;        // V_r, Qp x RP row-major, zero padded (state type)
    const void *Vhi;      // bf16 split of V (uint16, Qp x RP) for MODE_BF16X3
    const void *Vlo;
    const void *bcoef;    // b_i = sigma_i^2 / (beta + sigma_i^2), RP (state type)
    const void *Vu;       // fused kernel: per-chunk V operand blocks
    int r, RP, nchunk;
    Grid g;
    double tau, lam2, beta;   // tau = 1/(xi+beta), lam2 = 2*lambda (D^T D = 2L)
    const void *dprev;    // optional: d^k (for f^{k+1})
    void *fout;           // optional: f^{k+1}
    void *dout;           // optional: d^{k+1}
    int phase;            // shared launches: entry 2j + ((round + phase) & 1) is job j's
    const uint8_t *code;  // masked grids: per-voxel code (bit 7 inside, bits 0..2 inside
                          // face neighbours); NULL: the whole box
};

// Unfused reference kernels (any rank).
void launch_update_unfused(int mode, const IterArgs &a, hipStream_t s);
void launch_projw_unfused(int mode, const IterArgs &a, hipStream_t s);

// Fused single-pass iteration (MFMA contractions). One launch walks a table
// of bricks, each naming its job (an IterArgs entry), so one launch can cover
// many problems of one class (precision, padded rank, brick shape).
struct TileRef {
    int job, tx, ty, tz;   // brick (tx, ty, tz) of job `job`; bricks are 16 x ty x tz voxels
};
struct FusedShape {
    int ty, tz;
};
struct FusedLaunch {
    int mode, r, RP;
    FusedShape shape;
    const IterArgs *jobs;  // device array, two entries per job: [2j] for even, [2j+1] for odd k
    const TileRef *tiles;  // device array
    int ntiles;
    int round;             // iteration counter of the shared loop
    int maxchunk;          // largest chunk count among the jobs (0: unknown)
    double *mon;           // monitored iteration: per-brick sums of (z^{k+1} - z^k)^2
                           // (ntiles float64 slots), else NULL
};
// fused_supported(): whether (mode, padded rank, voxel count) has a fused kernel.
bool fused_supported(int mode, int RP, int64_t N);
bool launch_fused(const FusedLaunch &L, hipStream_t s);   // false: no such shape
FusedShape default_shape(int mode, const Grid &g);
std::vector<FusedShape> candidate_shapes(int mode, bool planar);
// Bricks of a grid in launch order for precision `mode`; with `code` only bricks
// holding an inside voxel.
void append_tiles(const Grid &g, int job, int mode, FusedShape sh, std::vector<TileRef> &out,
                  const std::vector<uint8_t> *code = nullptr);
// Per-chunk V operand blocks of the fused kernel (IterArgs::Vu points to them).
// `tail`: the kernel takes y of ranks 16..19 on the vector ALU (fused_tail()).
void fused_operands(const std::vector<double> &Vh, int Qp, int RP, bool f64_rows, bool tail,
                    std::vector<double> &Vop);
// Whether the fused kernel for (mode, RP, r) computes ranks 16..19 of y on the
// vector ALU: float32 with 17 <= r <= 20 (the u K-step bucket of 5).
inline bool fused_tail(int mode, int RP, int r) {
    return mode == MODE_FP32 && RP == 32 && r > 16 && r <= 20;
}
void fused_operands_bf16(const std::vector<double> &Vh, int Qp, int RP, std::vector<uint16_t> &Vop);

// Small problems split over spectral chunks (kernels_split.hip): one workgroup
// per (brick, chunk). The r-vectors travel as partial products: pin holds the
// per-chunk partials of y^k ([chunk][rank][voxel], RP x N per chunk), sin
// s^k = y^{k-1} + w^{k-1} (RP x N); the launch writes its chunks' partials of
// y^{k+1} to pout and, from the chunk-0 workgroups, s^{k+1} = y^k + w^k to sout.
struct SplitArgs {
    IterArgs a;
    const void *pin;
    void *pout;
    const void *sin;
    void *sout;
};
bool launch_split(int mode, const SplitArgs &sa, FusedShape sh, const TileRef *tiles, int ntiles,
                  hipStream_t s);   // false: no such mode or shape

// f and d around a fused iteration (see kernels_common.hip):
// pre: t = z^k + V_r w^k and, if f != NULL, f = t - dprev / beta (dprev NULL: d^k = 0;
// f may alias dprev); post: t <- beta (t - z^{k+1}) = d^{k+1}.
void launch_aux_pre(int mode, const IterArgs &a, void *t, void *f, const void *dprev,
                    hipStream_t s);
// Warm start: z^0 (and d^0 into dc when given) from voxel-major float64 inputs
// (NULL: zeros) into the chunked state, y^0 = V_r^T z^0 and w^0 = a.h - b.(y^0 -
// V_r^T d^0 / beta) into a.y, a.w (ranks below r), after the projection set a.h;
// V64: V_r in float64, Qp x RP.
void launch_warm(int mode, const IterArgs &a, const double *z0, const double *d0, const double *V64,
                 void *zc, void *dc, int Q, hipStream_t s);
void launch_aux_post(int mode, void *t, const void *znew, double beta, size_t count,
                     hipStream_t s);

// Data projection t = U_r^T m, ah = a .* (sigma .* t), w = ah, y = 0,
// mperp2 = ||m||^2 - ||t||^2; sets *bad != 0 if m holds a NaN/Inf.
// Outside voxels of a masked grid (code != NULL) get zeros and their data is not read.
void launch_project(int mode, const void *M, int P, const double *Ur, const double *sig,
                    const double *acoef, int r, int RP, int64_t N, double *t,
                    double *mperp2, void *ah, void *w, void *y, int *bad,
                    const uint8_t *code, hipStream_t s);

// Monitoring: per-block float64 partial sums of the objective terms, then a
// fixed-order final reduction into out[ST_COUNT].
struct MonArgs {
    const void *z;            // the iterate (state type; chunked, or voxel-major when ld > 0)
    const void *zprev;        // the iterate before it (same layout), or NULL
    const void *f;            // f of the same iteration (chunked state layout), or NULL
    const double *fstar;      // reference map for DFCS (N x Q float64, voxel-major), or NULL
    const double *V64;        // V_r in float64, (16 nchunk) x RP, zero padded
    const void *y;            // y = V_r^T z as the iteration left it (state type, RP x N
                              // rank-major, or voxel-major rows of yld), or NULL: the
                              // monitor contracts V64 with z
    int64_t yld;              // > 0: y voxel-major, element (r, n) at n yld + r
    const void *ypart;        // or y as npart per-chunk partial products (state type, each
    int npart;                // RP x N rank-major, RP N apart), summed in chunk order
    const double *dzpart;     // per-brick sums of (z - zprev)^2 from the iteration, or NULL
    int ndz;
    const double *sig, *t, *mperp2;   // singular values (RP), U_r^T m (r x N), ||m_perp||^2 (N)
    int r, RP, nchunk, Q;
    int64_t ld;               // voxel-major row length (0: chunked layout)
    Grid g;
    const uint8_t *code;      // mask codes or NULL
};
constexpr int kMonitorBlocks = 4096;  // partial sums: kMonitorBlocks x ST_COUNT doubles
constexpr int kMonitorSpreadTiles = 1024;  // grids of at most this many 16-voxel tiles: a block per tile
void launch_monitor(int mode, const MonArgs &a, double *partial, double *out, hipStream_t s);
int monitor_blocks(int64_t N);

// Chunked state -> voxel-major output (element type of the mode's I/O, or
// float64 when to_double is set).
void launch_output(int mode, const void *z, void *F, int Q, int64_t N, bool to_double,
                   hipStream_t s);

// ---- host-side plan rules shared by the solver and the server
constexpr double kEpsXi = 1e-10;      // epsilon of Eq. (sigma_cond)
constexpr double kXiFactor = 0.75;    // xi_p > 0.75 lambda ||D^T D|| (Sec. III-F)
constexpr double kRankTol = 5e-5;     // 0.005 % Frobenius error (Sec. III-F)

// Rank rule of Sec. III-F: rank > 0 is taken as given, -1 means min(P, Q),
// 0 the smallest r with ||K - K_r||_F < kRankTol ||K||_F (strict).
int rank_rule(const std::vector<double> &s, int rank);
// ||D^T D||_2 of the face-neighbour box grid with free boundary (D^T D = 2L).
double dtd_norm_closed(const Grid &g);

// Solve constants of one (dictionary, precision, rank, beta): float64 copies
// (V_r padded to Qp x RP, U_r P x r, singular values and a_i padded to RP)
// and byte images in the mode's state type (V, b_i, fused V operand blocks;
// Vop is empty unless `fused`).
struct HostConsts {
    std::vector<double> Vh, Ur, sig, a;
    std::vector<uint8_t> V, b, Vop;
};
void host_consts(int mode, const std::vector<double> &U, const std::vector<double> &s,
                 const std::vector<double> &V, int kmin, int P, int Q, int Qp, int r, int RP,
                 double beta, bool fused, HostConsts &out);

// ---- masked voxel sets (mask.cpp)
// Code bytes of a mask (N bytes, nonzero = inside) and the inside count.
void mask_codes(const Grid &g, const uint8_t *mask, std::vector<uint8_t> &code, int64_t &inside);
// ||D^T D||_2 of the graph of inside face neighbours (Lanczos, float64).
double masked_dtd_norm(const Grid &g, const std::vector<uint8_t> &code);
bool brick_has_inside(const Grid &g, const std::vector<uint8_t> &code, int64_t x0, int64_t y0,
                      int64_t z0, int tx, int ty, int tz);

// ---- exact-rank GEMM path (kernels_gemm.hip); voxel-major padded layouts
// Products C[n][m] = sum_k A[m][k] B[n][k] (A: M x K, row-major, float32 or
// bf16 operands, float32 accumulation), M a multiple of 128, K of 16 (float32)
// or 3 x 64 (bf16); false when the shape is not supported. float32: B is N x K.
// bf16 (split precision): B holds 2K/3 values per row (hi | lo) and column k
// reads column k mod 2K/3, so the third K segment is the hi half again. C is not
// stored: the u product (M = Qg) applies the z-update to it (z -> zn, and
// zn's hi/lo bf16 split into zs when zs is not null), the y product (M = Rg) the
// r-vector recursion with s = y + w (s in place; w^{k+1} into w, or its split
// into ws when ws is not null).
bool launch_gemm_u(bool bf16, const void *A, const void *B, int K, const float *z, float *zn,
                   uint16_t *zs, Grid g, int Qg, double tau, double lam2, double beta,
                   const uint8_t *code, hipStream_t s);
bool launch_gemm_y(bool bf16, const void *A, const void *B, int K, int64_t N, int Rg, const float *ah,
                   float *sv, float *w, uint16_t *ws, const float *bcoef, hipStream_t s);
void launch_gemm_from_ranks(const float *src, int RP, float *dst, uint16_t *ds, int64_t N, int Rg,
                            hipStream_t s, int nseg = 2);
// The same epilogues as separate passes over a product left in memory by a library
// GEMM (U: N x Qg, Y: N x Rg, voxel-major); splits are written hi | lo | hi.
void launch_epi_z(const float *U, const float *z, float *zn, uint16_t *zs3, Grid g, int Qg, double tau,
                  double lam2, double beta, const uint8_t *code, hipStream_t s);
void launch_epi_w(const float *Y, int64_t N, int Rg, const float *ah, float *sv, float *w, uint16_t *ws3,
                  const float *bcoef, hipStream_t s);
// f^{k+1} (into f, over dprev in place; f NULL: none) and d^{k+1} (into d) of the
// library path's iteration k from z^k, its u^k and z^{k+1} (voxel-major, count
// entries); dprev NULL: d^k = 0.
void launch_gemm_aux(const float *z, const float *u, const float *zn, const float *dprev, float *f,
                     float *d, size_t count, double beta, hipStream_t s);
// Library product (hipBLASLt): C[n][m] = sum_k A[m][k] B[n][k] for m < M, n < N,
// k < K; A M x K and B N x K row-major, bf16 or float32, C float32 (N x M).
// false when the library offers no algorithm for the shape.
struct LibGemm;
LibGemm *libgemm_create();
void libgemm_destroy(LibGemm *g);
bool libgemm_tn(LibGemm *g, bool bf16, const void *A, const void *B, float *C, int M, int64_t N, int K,
                hipStream_t s);
void launch_gemm_output(const float *z, void *F, bool to_double, int64_t N, int Q, int Qg,
                        hipStream_t s);

// ---- allocation-free solves (kernels_common.hip)
// Bytes of the static device array that an allocation-free solve takes its
// device memory from (the SSMAP_NOALLOC_MAX_BYTES of the C ABI).
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
// Device address of the current device's copy of that array (hipGetSymbolAddress
// once per device, then cached); the HIP error of the lookup otherwise.
hipError_t scratch_device_ptr(void **out);

// Fill a device array of `count` elements of `elem_bytes` (4 or 8) with zero.
void launch_zero(void *p, size_t count, int elem_bytes, hipStream_t s);

// float -> bf16 (round to nearest even) hi/lo split of V on the device.
void launch_split_bf16(const float *V, uint16_t *hi, uint16_t *lo, size_t count,
                       hipStream_t s);

}  // namespace ssmap
