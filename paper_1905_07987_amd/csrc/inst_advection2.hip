// Kernel instantiations for Advection<2>, orders 1..7.
#include "kernels.hpp"

namespace adg {

const KernelSet* kernels_advection2(int order) {
  switch (order) {
    case 1: return Launch<Advection<2>, 1>::set();
    case 2: return Launch<Advection<2>, 2>::set();
    case 3: return Launch<Advection<2>, 3>::set();
    case 4: return Launch<Advection<2>, 4>::set();
    case 5: return Launch<Advection<2>, 5>::set();
    case 6: return Launch<Advection<2>, 6>::set();
    case 7: return Launch<Advection<2>, 7>::set();
    default: return nullptr;
  }
}

int max_order_advection2() { return 7; }

}  // namespace adg
