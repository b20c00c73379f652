// Sweep and exact NNLS kernels for ranks padded to 64.
#include "nnls_exact.h"

template struct nmf::sweep::Launch<64>;
