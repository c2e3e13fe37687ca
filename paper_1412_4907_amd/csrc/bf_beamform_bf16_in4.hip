// Beamform kernel instantiations for one storage precision and input format (bf16, 4-bit input).
#include "bf_internal.h"
#include "bf_beamform.inc"

namespace bf {
template hipError_t launch_prec_in<2, true>(int, bool, Tile, const Launch&, int, size_t,
                                             hipStream_t);
template hipError_t launch_multi_in<2, true>(int, const Launch&, const Launch*, int, size_t,
                                              hipStream_t, int*, bool);
}
