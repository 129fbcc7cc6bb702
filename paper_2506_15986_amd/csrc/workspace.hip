// Workspace sizing for every operation (caller-allocated scratch).
#include "internal.h"

using namespace ann;

extern "C" size_t ann_workspace_size(int32_t op, int64_t n, int32_t dim, int32_t p0, int32_t p1)
{
    (void)dim;
    switch (op) {
    case ANN_OP_SEARCH:
        return search_ws_bytes(p0);
    case ANN_OP_BUILD_GRAPH:
        return build_graph_ws(n, dim, p0, p1);
    case ANN_OP_GT_KNN:
        return knn_workspace(n, p0, dim, p1);
    case ANN_OP_SELECT_HUBS:
        return select_hubs_ws(n, dim, p0);
    case ANN_OP_HUB_FEATURES:
        return hub_features_ws(n, p0);
    default:
        break;
    }
    (void)n;
    (void)p0;
    (void)p1;
    return 0;
}
