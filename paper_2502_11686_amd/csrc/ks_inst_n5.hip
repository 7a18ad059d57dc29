// ks_inst_n5.hip -- kernel instantiations for n = 5: wavefront family, with
// the MFMA backward and the unstaged level 0 as tunable variants.
#include "ks_device_blk.h"

namespace ks {

// host-only table (a function-local static is never emitted for the device)
const KernelSetList &list_n5() {
    static const KernelSet sets[] = {
    KS_SETS(5),
    };
    static const KernelSetList list = {sets, sizeof(sets) / sizeof(sets[0])};
    return list;
}

}  // namespace ks
