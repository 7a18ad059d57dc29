// ks_inst_blk_n48.hip -- workgroup-family kernel instantiations for n = 48.
#include "ks_device_mf.h"

namespace ks {

// host-only table (a function-local static is never emitted for the device)
const KernelSetList &list_blk_n48() {
    static const KernelSet sets[] = {
    KS_BLK_SETS_ONE(48),  // one record per workgroup: a record takes a wavefront per row tile
    KS_MF_SETS(48),       // forward variant 1: MFMA forward
    KS_OCC_SETS(48),  // forward variant 2: 2-D tiled forward at the other occupancy target
    };
    static const KernelSetList list = {sets, sizeof(sets) / sizeof(sets[0])};
    return list;
}

}  // namespace ks
