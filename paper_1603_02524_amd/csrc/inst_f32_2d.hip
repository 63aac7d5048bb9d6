// Kernel instantiations for float vectors in 2D.
#include "dispatch.hpp"

namespace dgmg {
template struct Kern<float, 2>;
}
