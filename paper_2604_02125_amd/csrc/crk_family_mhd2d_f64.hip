// Instances of the cRKFR kernels for one family: double, EQ_MHD, dim 2.
#include "crk_family_impl.hpp"
template struct crk::Family<double, crk::EQ_MHD, 2>;
