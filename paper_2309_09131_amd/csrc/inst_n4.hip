// Kernels for 4-mode tensors.
#define NM 4
#include "inst.hpp"
