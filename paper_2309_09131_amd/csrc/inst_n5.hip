// Kernels for 5-mode tensors.
#define NM 5
#include "inst.hpp"
