// Kernel instantiations for Euler<3>, orders 1..5.
#include "kernels.hpp"

namespace adg {

const KernelSet* kernels_euler3(int order) {
  switch (order) {
    case 1: return Launch<Euler<3>, 1>::set();
    case 2: return Launch<Euler<3>, 2>::set();
    case 3: return Launch<Euler<3>, 3>::set();
    case 4: return Launch<Euler<3>, 4>::set();
    case 5: return Launch<Euler<3>, 5>::set();
    default: return nullptr;
  }
}

int max_order_euler3() { return 5; }

}  // namespace adg
