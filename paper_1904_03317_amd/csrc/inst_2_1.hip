// Kernel instantiation for dim 2, degree 1.
#include "inst.hpp"
GMG_INSTANTIATE(2, 1)
