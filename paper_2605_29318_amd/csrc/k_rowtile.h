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
    const float *v32 = nullptr;      // [entries][8]: H of rows 0..3, M of rows 0..3 (FP32 copies)
    const double *v64 = nullptr;     // [entries][8] (FP64)
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
// HY = H Y alone, for the preconditioner: FP32 accumulation on the FP32 copy,
// FP64 on the FP64 copy.
int spmm_h32(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const float *Y, int64_t ldy, float *HY,
             int64_t ldo, const int *row_obj, const int *status);
int spmm_h64(ff_ctx *ctx, hipStream_t st, const RTView &v, int sub, int m, const double *Y, int64_t ldy, double *HY,
             int64_t ldo, const int *row_obj, const int *status);

}  // namespace rt
}  // namespace ff
