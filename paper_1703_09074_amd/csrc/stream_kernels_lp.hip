// Streaming contractions with 16-bit matrix-core operands (bfloat16 or
// float16, rounded to nearest even from the float32 tiles in LDS; float32
// accumulation): the precision variant of the sketch, power-iteration and
// mode-product kernels.

#include "stream_tiles.h"

namespace rcp {

hipError_t launch_contract_out_lp(int precision, const StreamGeom& g, int l, const float* Z,
                                  uint64_t seed, uint32_t tag, int okind, float* part, int P,
                                  double* sq_part, hipStream_t s, int mb_cap) {
    if (precision == kPrecBf16) return launch_contract_out_t<kPrecBf16>(g, l, Z, seed, tag, okind, part, P, sq_part, s, mb_cap);
    if (precision == kPrecFp16) return launch_contract_out_t<kPrecFp16>(g, l, Z, seed, tag, okind, part, P, sq_part, s, mb_cap);
    return hipErrorInvalidValue;
}

hipError_t launch_power_fused_lp(int precision, const StreamGeom& g, int l, const float* Qt,
                                 float* part, int P, hipStream_t s) {
    if (precision == kPrecBf16) return launch_power_fused_t<kPrecBf16>(g, l, Qt, part, P, s);
    if (precision == kPrecFp16) return launch_power_fused_t<kPrecFp16>(g, l, Qt, part, P, s);
    return hipErrorInvalidValue;
}

hipError_t launch_contract_in_lp(int precision, const StreamGeom& g, int l, const float* Qpadded,
                                 int lout, float* out, int P, hipStream_t s) {
    if (precision == kPrecBf16) return launch_contract_in_t<kPrecBf16>(g, l, Qpadded, lout, out, P, s);
    if (precision == kPrecFp16) return launch_contract_in_t<kPrecFp16>(g, l, Qpadded, lout, out, P, s);
    return hipErrorInvalidValue;
}

hipError_t launch_sketch_group_lp(const SketchDesc* d, int count, int gx, int gy, int NB, int MB,
                                  bool caseB, bool stored, int precision, hipStream_t s) {
    if (precision == kPrecBf16) return launch_sketch_group_t<kPrecBf16>(d, count, gx, gy, NB, MB, caseB, stored, s);
    if (precision == kPrecFp16) return launch_sketch_group_t<kPrecFp16>(d, count, gx, gy, NB, MB, caseB, stored, s);
    return hipErrorInvalidValue;
}

hipError_t launch_power_group_lp(const PowerDesc* d, int count, int gx, int NB, int MB, bool fused,
                                 bool caseB, int precision, hipStream_t s) {
    if (precision == kPrecBf16) return launch_power_group_t<kPrecBf16>(d, count, gx, NB, MB, fused, caseB, s);
    if (precision == kPrecFp16) return launch_power_group_t<kPrecFp16>(d, count, gx, NB, MB, fused, caseB, s);
    return hipErrorInvalidValue;
}

}  // namespace rcp
