// Kernels for 8-mode tensors.
#define NM 8
#include "inst.hpp"
