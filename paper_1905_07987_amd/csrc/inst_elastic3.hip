// Kernel instantiations for Elastic3, orders 1..4.
#include "kernels.hpp"

namespace adg {

const KernelSet* kernels_elastic3(int order) {
  switch (order) {
    case 1: return Launch<Elastic3, 1>::set();
    case 2: return Launch<Elastic3, 2>::set();
    case 3: return Launch<Elastic3, 3>::set();
    case 4: return Launch<Elastic3, 4>::set();
    default: return nullptr;
  }
}

int max_order_elastic3() { return 4; }

}  // namespace adg
