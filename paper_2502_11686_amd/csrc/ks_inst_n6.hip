// ks_inst_n6.hip -- kernel instantiations for n = 6: wavefront-family forward
// with the workgroup-family (MFMA) backward, which is faster here than the
// wavefront-family backward.
#include "ks_device_blk.h"

namespace ks {

// host-only table (a function-local static is never emitted for the device)
const KernelSetList &list_n6() {
    static const KernelSet sets[] = {
    KS_HYB_SETS(6),
    };
    static const KernelSetList list = {sets, sizeof(sets) / sizeof(sets[0])};
    return list;
}

}  // namespace ks
