// Kernel instantiation for dim 3, degree 4.
#include "inst.hpp"
GMG_INSTANTIATE(3, 4)
