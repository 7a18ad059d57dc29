// ks_inst_n4.hip -- kernel instantiations for one group of state dimensions.
#include "ks_device.h"

namespace ks {

// host-only table (a function-local static is never emitted for the device)
const KernelSetList &list_n4() {
    static const KernelSet sets[] = {
    KS_SETS(4),
    };
    static const KernelSetList list = {sets, sizeof(sets) / sizeof(sets[0])};
    return list;
}

}  // namespace ks
