// Kernel instantiation for dim 3, degree 2.
#include "inst.hpp"
GMG_INSTANTIATE(3, 2)
