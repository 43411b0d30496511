// Step kernels of space order 16 (half-width 8): every block shape, plain
// and imaging steps, the batch kernel and the persistent kernel.
#include "wave_step.h"

template struct wave::OrderOps<16>;
