// Row-tile copy of the fused [H, M] CSR for the SpMM of the eigensolver.
//
// Rows are grouped in tiles of four consecutive (cell-sorted, so spatially
// close) rows. A tile stores the union of its rows' column lists, ascending,
// and for every union entry the four H values and the four M values of its
// rows (zero where a row lacks the column). The SpMM then gathers each block
// row Y_j once per tile instead of once per row: neighbouring RKPM rows share
// most of their columns, so the gathered bytes drop to well under half for
// about a tenth more matrix bytes.
#pragma once

#include "ff_internal.h"

namespace ff {
namespace rt {

constexpr int kTileRows = 4;

struct RTView {
    int64_t n = 0, ntiles = 0, entries = 0;
    const int64_t *tptr = nullptr;   // [ntiles + 1]
    const int32_t *tcol = nullptr;   // [entries]
    const float *v32 = nullptr;      // [2][entries][4]: H of rows 0..3 per entry, then M likewise (FP32 copies)
    const double *v64 = nullptr;     // [2][entries][4] (FP64)
};

// Build the tile structure and the value copies asked for (want32 / want64)
// into the context's workspace slots; synchronises the stream once (the
// number of union entries sizes the arrays).
int build_ws(ff_ctx *ctx, hipStream_t st, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
             const double *M, int want32, int want64, RTView *out);

// [HY, MY] = [H, M] Y on the tile copy; sub selects a launch shape (0..kSubs-1).
constexpr int kSubs = 3;
extern const char *kSubNames[kSubs];
int spmm32(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const float *Y, int64_t ldy, float *HY,
           float *MY, int64_t ldo, const int *row_obj, const int *status);
int spmm64(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const double *Y, int64_t ldy, double *HY,
           double *MY, int64_t ldo, const int *row_obj, const int *status);
// One step of the Chebyshev-Jacobi preconditioner fused into the H-only
// product of DZ (rows of object o use coef[o * stride + 2 step - 1] = f1 and
// coef[o * stride + 2 step] = f2): R -= D^-1 H DZ, DZ' = f1 DZ + f2 R, W += DZ'.
// R, DZ and dz_out share the leading dimension of DZ; dz_out must not alias DZ
// (other tiles still gather it).
template <typename T> struct ChebStep {
    const double *coef = nullptr;
    int stride = 0, step = 0;
    const T *dinv = nullptr;
    T *R = nullptr, *dz_out = nullptr, *W = nullptr;
    int64_t ldw = 0;
};
int cheb_step32(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const float *DZ, int64_t ld,
                const int *row_obj, const int *status, const ChebStep<float> &cs);
int cheb_step64(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const double *DZ, int64_t ld,
                const int *row_obj, const int *status, const ChebStep<double> &cs);

// H-only FP32 copy in tiles of eight rows (the preconditioner's products):
// vh[entry][8] holds the H values of the tile's eight rows.
constexpr int kTile8 = 8;
constexpr int kHSubs = 3;            // launch shapes of the H-only kernels
struct RT8View {
    int64_t n = 0, ntiles = 0, entries = 0;
    const int64_t *tptr = nullptr;   // [ntiles + 1]
    const int32_t *tcol = nullptr;   // [entries]
    const float *vh = nullptr;       // [entries][8]
    const float *vm = nullptr;       // [entries][8] M values, when built with M
    // FP16 copy of H scaled by 2^e (largest magnitude in [2^14, 2^15)); hscale = 2^-e. When present the
    // H-only products (spmm_h_t8, cheb_step_t8) read it instead of vh
    const uint16_t *vh16 = nullptr;  // [entries][8] binary16 bits
    float hscale = 1.f;
    // the zero-free copy of (vh, vm) (build_t8z_ws): per entry a byte mask of the rows present (H or
    // M not +-0), and their (H, M) pairs in entry and row order, each tile's from pair poff[t] on
    const uint8_t *m8 = nullptr;     // [entries]
    const int64_t *poff = nullptr;   // [ntiles + 1]
    const float *pv = nullptr;       // [2 * pairs + 16]
};
int build_t8_ws(ff_ctx *ctx, hipStream_t st, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
                RT8View *out, const double *M = nullptr);
// adds the FP16 copy of vh to a built view (vh16 storage: entries * 8 halves at out16, or the workspace)
int build_t8_half(ff_ctx *ctx, hipStream_t st, RT8View *v, uint16_t *out16 = nullptr);
// block widths the eight-row kernels take: m % 8 == 0, 8 <= m <= 64, 16-byte aligned rows
bool t8_ok(int m, int64_t ldy, int64_t ldo);
int spmm_h_t8(ff_ctx *ctx, hipStream_t st, const RT8View &v, int sub, int m, const float *Y, int64_t ldy, float *HY,
              int64_t ldo, const int *row_obj, const int *status);
int cheb_step_t8(ff_ctx *ctx, hipStream_t st, const RT8View &v, int sub, int m, const float *DZ, int64_t ld,
                 const int *row_obj, const int *status, const ChebStep<float> &cs);

// The preconditioner's Chebyshev step on the matrix cores: H of the eight-row
// tiles in binary16 (scaled by 2^e as vh16), cut into K-blocks of 16 union
// entries, vq[kblock][8 rows][16 entries] (zero past a tile's last entry), and
// the iterate DZ in binary16, [rows][m]; products accumulate in FP32 on
// v_mfma_f32_16x16x16_f16.
// K-blocks per group of the zero-free copy (the K-blocks one super-block of the kernel multiplies)
constexpr int kTqPackGroup = 4;
struct RTQView {
    int64_t n = 0, ntiles = 0, nkb = 0;
    const int64_t *tptr = nullptr;   // [ntiles + 1] union entries of the eight-row copy
    const int32_t *tcol = nullptr;   // [entries]
    const int64_t *kptr = nullptr;   // [ntiles + 1] first K-block of each tile
    const uint16_t *vq = nullptr;    // [nkb][8][16] binary16 bits
    float hscale = 1.f;              // 2^-e
    // the same K-blocks without their zeros (build_tq_pack): per K-block a 128-bit mask of the
    // values present, bit 16 r + e for row r and entry e (two words: rows 0-3, rows 4-7), and the
    // present values in that bit order, each tile's from pvoff[t] on, each group of kTqPackGroup
    // consecutive K-blocks of a tile starting at a multiple of eight halves (zeros between); the
    // kernels expand them into the K-block's fragments in registers (the same operands, so the
    // same sums bit for bit)
    const uint64_t *pmask = nullptr; // [nkb][2]
    const int64_t *pvoff = nullptr;  // [ntiles + 1], multiples of 8
    const uint16_t *pval = nullptr;  // [pvoff[ntiles] + 8] binary16 bits (8 halves of padding)
};
// builds the K-blocked copy from the FP32 values of a built eight-row copy into workspace slots;
// build_tq_ptr (tile K-block pointers kptr[ntiles + 1], cnt[ntiles + 1] scratch, their total nkb)
// and build_tq_fill (nkb * 128 binary16 values) do the same into the caller's storage
int build_tq(ff_ctx *ctx, hipStream_t st, const RT8View &v8, RTQView *out);
int build_tq_ptr(ff_ctx *ctx, hipStream_t st, const RT8View &v8, int64_t *kptr, int64_t *cnt, int64_t *nkb);
int build_tq_fill(ff_ctx *ctx, hipStream_t st, const RT8View &v8, const int64_t *kptr, int64_t nkb, uint16_t *vq,
                  RTQView *out);
// the zero-free copy of a built K-blocked copy: pmask [nkb][2] and pvoff [ntiles + 1] from the
// caller (cnt [ntiles + 1] scratch), pval allocated by alloc(bytes) once the count is known
// (returns nullptr on failure)
int build_tq_pack(ff_ctx *ctx, hipStream_t st, RTQView *v, uint64_t *pmask, int64_t *pvoff, int64_t *cnt,
                  void *(*alloc)(void *, size_t), void *alloc_arg);
// the same into workspace slots
int build_tq_pack_ws(ff_ctx *ctx, hipStream_t st, RTQView *v);
// block widths the matrix-core kernels take: m in {32, 64}
bool tq_ok(int m);
// one Chebyshev step, binary16 iterate: R -= D^-1 H DZ, DZ' = f1 DZ + f2 R (stored in binary16),
// and by wmode: 1 W += DZ', 0 W untouched, 2 W += DZ + DZ' (the previous step's DZ' with this one's,
// so that W is read and written every other step); DZ and dz_out are [rows][m], R has leading
// dimension m, W ldw
struct ChebStepQ {
    const double *coef = nullptr;
    int stride = 0, step = 0;
    const float *dinv = nullptr;
    float *R = nullptr, *W = nullptr;
    uint16_t *dz_out = nullptr;
    int64_t ldw = 0;
    int wmode = 1;
};
// sub selects a launch shape (waves per block, K-blocks in flight), 0 .. kTqSubs - 1; shapes
// kTqPacked and above read the zero-free copy (pmask, pval)
constexpr int kTqSubs = 15;
constexpr int kTqPacked = 8;
int cheb_step_tq(ff_ctx *ctx, hipStream_t st, const RTQView &v, int sub, int m, const uint16_t *DZ,
                 const int *row_obj, const int *status, const ChebStepQ &cs);
// HY = H Y (Y binary16 [rows][m], HY FP32 with leading dimension ldo)
int spmm_h_tq(ff_ctx *ctx, hipStream_t st, const RTQView &v, int sub, int m, const uint16_t *Y, float *HY,
              int64_t ldo);

// H-only FP32 copy in tiles of sixteen rows, for the MFMA form of the
// preconditioner's products: vh[entry][16].
constexpr int kTile16 = 16;
struct RT16View {
    int64_t n = 0, ntiles = 0, entries = 0;
    const int64_t *tptr = nullptr;   // [ntiles + 1]
    const int32_t *tcol = nullptr;   // [entries]
    const float *vh = nullptr;       // [entries][16]
};
int build_t16_ws(ff_ctx *ctx, hipStream_t st, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *H,
                 RT16View *out);
// block widths the sixteen-row kernels take: m in {4, 8, 12, 16, 32, 64}, 16-byte aligned rows
bool t16_ok(int m, int64_t ldy, int64_t ldo);
int spmm_h_t16(ff_ctx *ctx, hipStream_t st, const RT16View &v, int sub, int m, const float *Y, int64_t ldy, float *HY,
               int64_t ldo, const int *row_obj, const int *status);
int cheb_step_t16(ff_ctx *ctx, hipStream_t st, const RT16View &v, int sub, int m, const float *DZ, int64_t ld,
                  const int *row_obj, const int *status, const ChebStep<float> &cs);

// [HY, MY] = [H, M] Y (FP32 blocks, FP64 accumulation on FP64 MFMA) on an
// eight-row copy built with M; m in {4, 8, 12, 16, 32, 64}; sub 0 .. kHm8Subs - 1 (3, 4 and 6 take
// four-entry steps on the FP32 matrix cores, each added in FP64; 5, 6 and 7 pipeline the loads; 8 and 9
// read the zero-free copy; 10 chains four FP32 steps before each FP64 addition).
constexpr int kHm8Subs = 11;
bool hm8_ok(int m, int64_t ldy, int64_t ldo);
// builds the zero-free copy of a built eight-row [H, M] copy into workspace slots
int build_t8z_ws(ff_ctx *ctx, hipStream_t st, RT8View *v);
int spmm_hm8(ff_ctx *ctx, hipStream_t st, const RT8View &v, int sub, int m, const float *Y, int64_t ldy, float *HY,
             float *MY, int64_t ldo, const int *row_obj, const int *status);

// HY = H Y alone, for the preconditioner: FP32 accumulation on the FP32 copy,
// FP64 on the FP64 copy.
int spmm_h32(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const float *Y, int64_t ldy, float *HY,
             int64_t ldo, const int *row_obj, const int *status);
int spmm_h64(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const double *Y, int64_t ldy, double *HY,
             int64_t ldo, const int *row_obj, const int *status);

}  // namespace rt
}  // namespace ff
