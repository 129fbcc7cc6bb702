// Internal cross-file declarations of libann (sizes of composite workspaces).
#pragma once

#include "common.h"

namespace ann {

struct Carve {
    unsigned char *p;
    template <typename T> T *take(size_t count)
    {
        T *r = reinterpret_cast<T *>(p);
        p += round_up(count * sizeof(T), 256);
        return r;
    }
};

size_t knn_workspace(int64_t n, int64_t rows, int dim, int K);
size_t build_graph_ws(int64_t n, int dim, int K, int R);
size_t medoid_ws(int64_t n, int dim);
size_t select_hubs_ws(int64_t n, int dim, int nh);
size_t hub_features_ws(int64_t n, int nh);

}  // namespace ann
