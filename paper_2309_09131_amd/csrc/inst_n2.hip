// Kernels for 2-mode tensors.
#define NM 2
#include "inst.hpp"
