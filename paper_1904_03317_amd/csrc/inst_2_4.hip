// Kernel instantiation for dim 2, degree 4.
#include "inst.hpp"
GMG_INSTANTIATE(2, 4)
