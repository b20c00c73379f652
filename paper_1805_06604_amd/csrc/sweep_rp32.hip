// Sweep kernels for ranks padded to 32.
#include "sweep_impl.h"

template struct nmf::sweep::Launch<32>;
