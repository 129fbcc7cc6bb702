// Workspace sizing for every operation (caller-allocated scratch).
#include "common.h"

extern "C" size_t ann_workspace_size(int32_t op, int64_t n, int32_t dim, int32_t p0, int32_t p1)
{
    (void)dim;
    switch (op) {
    case ANN_OP_SEARCH:
        return 256;
    default:
        break;
    }
    (void)n;
    (void)p0;
    (void)p1;
    return 0;
}
