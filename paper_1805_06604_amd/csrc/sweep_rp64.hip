// Sweep kernels for ranks padded to 64.
#include "sweep_impl.h"

template struct nmf::sweep::Launch<64>;
