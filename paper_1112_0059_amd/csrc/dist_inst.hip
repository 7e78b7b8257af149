// One translation unit per (operand format, list length): the K1 variants
// of dist_topk.h for LNBNN_OP / LNBNN_KP, exposed as LNBNN_SYM(v).  The
// build compiles this file once per entry of LNBNN_DIST_INSTANCES, so the
// instances compile in parallel.
#include "dist_topk.h"

#if !defined(LNBNN_OP) || !defined(LNBNN_KP) || !defined(LNBNN_SYM)
#error "dist_inst.hip is compiled with -DLNBNN_OP=<policy> -DLNBNN_KP=<length> -DLNBNN_SYM=<name>"
#endif

namespace lnbnn {

void *LNBNN_SYM(int v) { return pick_variant<LNBNN_OP, LNBNN_KP>(v); }

}  // namespace lnbnn
