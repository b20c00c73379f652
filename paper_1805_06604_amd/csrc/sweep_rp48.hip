// Sweep kernels for ranks padded to 48.
#include "sweep_impl.h"

template struct nmf::sweep::Launch<48>;
