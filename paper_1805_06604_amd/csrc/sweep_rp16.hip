// Sweep kernels for ranks padded to 16.
#include "sweep_impl.h"

template struct nmf::sweep::Launch<16>;
