// ks_inst_n1_3.hip -- kernel instantiations for one group of state dimensions.
#include "ks_device.h"

namespace ks {

// host-only table (a function-local static is never emitted for the device)
const KernelSetList &list_n1_3() {
    static const KernelSet sets[] = {
    make_set<1, 1>(),
    make_set<1, 2>(),
    make_set<2, 1>(), make_set<2, 2>(), make_set<2, 4>(),
    make_set<3, 2>(), make_set<3, 3>(), make_set<3, 6>(),
    };
    static const KernelSetList list = {sets, sizeof(sets) / sizeof(sets[0])};
    return list;
}

}  // namespace ks
