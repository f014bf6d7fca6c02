// Kernels for 7-mode tensors.
#define NM 7
#include "inst.hpp"
