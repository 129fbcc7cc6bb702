// Internal interface of the exact kNN engines (knn.hip).
#pragma once

#include "common.h"

namespace ann {

namespace knn {
struct Ent;
}

struct KnnArgs {
    const float *base;
    int64_t n;
    int dim;
    const float *queries;
    int64_t rows;
    int K;
    int exclude_self;
    const int32_t *self_col;    // column excluded for query row g (null: column g)
    knn::Ent *buf;
    int cap;
    int32_t *out_ids;
    float *out_f;
    double *out_d;
};

// Workspace bytes for knn_run.
size_t knn_workspace(int64_t n, int64_t rows, int dim, int K);

// Exact top-K by (squared L2, id) of `rows` query rows against `base`.
// force_engine: 0 = pick (int8 matrix cores when all values are integers in
// [0,255] and dim % 32 == 0, else FP64), 1 = int8 only, 2 = FP64 only.
// With exclude_self, query row g never returns base column self_col[g]
// (column g when self_col is null).  Synchronises `st`.
ann_status knn_run(const float *base, int64_t n, int dim, const float *queries, int64_t rows,
                   int K, bool exclude_self, int32_t *out_ids, float *out_f, double *out_d,
                   void *ws, size_t ws_bytes, hipStream_t st, int force_engine,
                   const int32_t *self_col = nullptr);

// Sets *result when every value of x[0..count) is an integer in [0,255].
ann_status data_is_uint8(const float *x, int64_t count, int *flag_dev, bool *result,
                         hipStream_t st);

}  // namespace ann
