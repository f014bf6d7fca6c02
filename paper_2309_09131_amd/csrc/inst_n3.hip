// Kernels for 3-mode tensors.
#define NM 3
#include "inst.hpp"
