// Kernels for 6-mode tensors.
#define NM 6
#include "inst.hpp"
