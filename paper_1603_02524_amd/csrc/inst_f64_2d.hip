// Kernel instantiations for double vectors in 2D.
#include "dispatch.hpp"

namespace dgmg {
template struct Kern<double, 2>;
}
