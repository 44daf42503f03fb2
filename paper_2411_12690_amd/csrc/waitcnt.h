// Explicit memory waits for the MFMA kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace mos {

// Wait for every outstanding memory operation of this wave (s_waitcnt
// vmcnt(0) lgkmcnt(0); loads through a generic pointer count in both, and
// vector stores count in vmcnt on this architecture).  The compiler's wait
// insertion merges control-flow paths that leave different numbers of
// operations outstanding (a conditional load, a conditional store)
// pessimistically: the next MFMA that reads an older load then waits for
// every later one too, including a prefetch issued for the next step.  A
// wait placed where only old operations are outstanding (the end of a rare
// branch, the top of a block after its predecessor's stores) removes that
// merge, so the waits inside the MFMA chain are exact again.
__device__ __forceinline__ void vm_wait_all() { __builtin_amdgcn_s_waitcnt(0x0070); }

}  // namespace mos
