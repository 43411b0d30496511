// Step kernels of space order 8 (half-width 4): every block shape, plain
// and imaging steps, the batch kernel and the persistent kernel.
#include "wave_step.h"

template struct wave::OrderOps<8>;
