// Kernel instantiations for float vectors in 3D.
#include "dispatch.hpp"

namespace dgmg {
template struct Kern<float, 3>;
}
