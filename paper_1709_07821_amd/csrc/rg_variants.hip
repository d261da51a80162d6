// rg_variants.hip - specialised variants for matched non-bitset pairs.
// Until a specialised kernel exists for a class, the class runs the generic
// LDS kernel, which computes the same result.
#include "rg_internal.h"

namespace rg {

void launch_aa(const ComputeArgs& a, hipStream_t st) { launch_generic(a, st); }
void launch_gallop(const ComputeArgs& a, hipStream_t st) { launch_generic(a, st); }
void launch_ab(const ComputeArgs& a, hipStream_t st) { launch_generic(a, st); }
void launch_rr(const ComputeArgs& a, hipStream_t st) { launch_generic(a, st); }

}  // namespace rg
