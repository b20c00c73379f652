// Sweep and exact NNLS kernels for ranks padded to 32.
#include "nnls_exact.h"

template struct nmf::sweep::Launch<32>;
