// Kernel instantiation for dim 3, degree 3.
#include "inst.hpp"
GMG_INSTANTIATE(3, 3)
