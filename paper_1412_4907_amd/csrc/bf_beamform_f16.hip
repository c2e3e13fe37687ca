// Beamform kernel instantiations for one storage precision and input format (f16, int8 input).
#include "bf_internal.h"
#include "bf_beamform.inc"

namespace bf {
template hipError_t launch_prec_in<1, false>(int, bool, Tile, const Launch&, int, size_t,
                                             hipStream_t);
template hipError_t launch_multi_in<1, false>(int, const Launch&, const Launch*, int, size_t,
                                              hipStream_t, int*, bool);
}
