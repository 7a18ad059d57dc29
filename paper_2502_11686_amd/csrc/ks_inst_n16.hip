// ks_inst_n16.hip -- kernel instantiations for one group of state dimensions.
#include "ks_device.h"

namespace ks {

// host-only table (a function-local static is never emitted for the device)
const KernelSetList &list_n16() {
    static const KernelSet sets[] = {
    make_set<16, 8>(),
    make_set<16, 16>(),
    };
    static const KernelSetList list = {sets, sizeof(sets) / sizeof(sets[0])};
    return list;
}

}  // namespace ks
