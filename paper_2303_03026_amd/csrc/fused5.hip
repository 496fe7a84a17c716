// The fused stage with three ghost layers: the HLL instances and the
// dispatch on the flux (the kernel is in fused5_stage.h; the HLLC and HLLD
// instances are built in fused5_hllc.hip and fused5_hlld.hip).
#include "fused5_stage.h"

namespace amrvac {

hipError_t launch_fused5_stage(hipStream_t s, const GridConst& G, const Tables& T, const JobScalars& J, const void* in,
                               const void* base, void* out, double w, const PhysConst& P, DevStatus* st,
                               double* part, void* freg, const JobCfl* cfl) {
  if (P.flux == FLUX_HLLC) return launch_fused5_hllc(s, G, T, J, in, base, out, w, P, st, part, freg, cfl);
  if (P.flux == FLUX_HLLD) return launch_fused5_hlld(s, G, T, J, in, base, out, w, P, st, part, freg, cfl);
  return launch_fused5_flux<FLUX_HLL>(s, G, T, J, in, base, out, w, P, st, part, freg, cfl);
}

}  // namespace amrvac
