// Kernel instantiations for Advection<3>, orders 1..6.
#include "kernels.hpp"

namespace adg {

const KernelSet* kernels_advection3(int order) {
  switch (order) {
    case 1: return Launch<Advection<3>, 1>::set();
    case 2: return Launch<Advection<3>, 2>::set();
    case 3: return Launch<Advection<3>, 3>::set();
    case 4: return Launch<Advection<3>, 4>::set();
    case 5: return Launch<Advection<3>, 5>::set();
    case 6: return Launch<Advection<3>, 6>::set();
    default: return nullptr;
  }
}

int max_order_advection3() { return 6; }

}  // namespace adg
