// Instances of the cRKFR kernels for one family: float, EQ_EULER, dim 2.
#include "crk_family_impl.hpp"
template struct crk::Family<float, crk::EQ_EULER, 2>;
