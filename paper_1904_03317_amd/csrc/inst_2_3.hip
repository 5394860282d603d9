// Kernel instantiation for dim 2, degree 3.
#include "inst.hpp"
GMG_INSTANTIATE(2, 3)
