// Kernel instantiation for dim 3, degree 1.
#include "inst.hpp"
GMG_INSTANTIATE(3, 1)
