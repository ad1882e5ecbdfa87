// Persistent 2D isotropic kernels with a zero LDS halo.
#include "fdw_iso2d_persist.h"

namespace fdw {

hipError_t launch_iso2d_persistent_halo(int R, const Persist2DArgs *one, const Geom &g, const Persist2DArgs *shots,
                                      int n, size_t lds, hipStream_t s, const LaunchEvents &ev) {
    return p2d_form_launch<true>(R, one, g, shots, n, lds, s, ev);
}

}  // namespace fdw
