// Workspace sizes of primitives that are not built yet.
#include "fg_common.h"
size_t fg_msbfs_workspace_bytes(const fg_graph*, int32_t) { return 0; }
