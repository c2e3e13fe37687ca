// Beamform kernel instantiations for one storage precision (bf16).
#include "bf_internal.h"
#include "bf_beamform.inc"

namespace bf {
template hipError_t launch_prec<2>(int, bool, Tile, const Launch&, int, size_t, hipStream_t);
template hipError_t launch_multi_prec<2>(int, const Launch&, const Launch*, int, size_t,
                                            hipStream_t, int*);
}
