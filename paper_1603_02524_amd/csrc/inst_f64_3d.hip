// Kernel instantiations for double vectors in 3D.
#include "dispatch.hpp"

namespace dgmg {
template struct Kern<double, 3>;
}
