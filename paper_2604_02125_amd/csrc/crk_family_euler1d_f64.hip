// Instances of the cRKFR kernels for one family: double, EQ_EULER, dim 1.
#include "crk_family_impl.hpp"
template struct crk::Family<double, crk::EQ_EULER, 1>;
