// ks_inst_n16.hip -- kernel instantiations for n = 16: the workgroup family
// (2-D tiled forward, MFMA backward), faster here than the wavefront family,
// whose 49-lane units leave a wavefront at one per SIMD by register use.
#include "ks_device_blk.h"

namespace ks {

// host-only table (a function-local static is never emitted for the device)
const KernelSetList &list_n16() {
    static const KernelSet sets[] = {
    KS_BLK_SETS(16),
    };
    static const KernelSetList list = {sets, sizeof(sets) / sizeof(sets[0])};
    return list;
}

}  // namespace ks
