// Kernel instantiation for dim 2, degree 2.
#include "inst.hpp"
GMG_INSTANTIATE(2, 2)
