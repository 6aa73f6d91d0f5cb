#include "api_internal.h"
namespace mrx {
size_t extra_workspace_bytes(mrx_plan_s* p) { (void)p; return 0; }
}
