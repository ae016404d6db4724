// Legendre synthesis and adjoint kernels of the 64-pair ring groups where only the north rings carry weight
// (one translation unit per class, compiled in parallel).
#include "akra_leg.h"

namespace akra {
template void leg_synth_cls<GCLS_NORTH>(Plan &, bool, int, const int *, int, int);
template int leg_adj_cls<GCLS_NORTH>(Plan &, bool, int, const int *, int, int, const uint8_t *, int, int);
}  // namespace akra
