// The fused stage with three ghost layers: the HLLD instances.
#include "fused5_stage.h"

namespace amrvac {

hipError_t launch_fused5_hlld(hipStream_t s, const GridConst& G, const Tables& T, const JobScalars& J,
                              const void* in, const void* base, void* out, double w, const PhysConst& P,
                              DevStatus* st, double* part, void* freg, const JobCfl* cfl) {
  return launch_fused5_flux<FLUX_HLLD>(s, G, T, J, in, base, out, w, P, st, part, freg, cfl);
}

}  // namespace amrvac
