// FDM local solves with the six tensor contractions on MFMA (BF16 / FP16 inputs,
// FP32 accumulation).  Placeholder until the matrix-core path lands.
#include "sem_internal.h"

namespace sem {

void launch_fdm_mfma(const Ctx &c, const Level &L, const float *r, float *z, bool asm_mode,
                     int prec, hipStream_t s) {
  (void)c; (void)L; (void)r; (void)z; (void)asm_mode; (void)prec; (void)s;
  fail(SEM_EUNSUPPORTED, "BF16/FP16 MFMA FDM is not available in this build");
}

}  // namespace sem
