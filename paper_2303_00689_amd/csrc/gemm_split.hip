// Split-precision MFMA GEMM (BF16 / FP16 hi-lo splits of FP32 storage, FP32
// accumulation).  Not enabled yet: every split mode reports an error.
#include "common.h"
namespace xl {
void gemm_split(const GemmArgs &, int, hipStream_t) {}
}
