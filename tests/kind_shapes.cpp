// kind_shapes.cpp -- prints the time-fused path's compile-time kind shapes
// (mech_internal.h) for tests/test_abi.py to check against the binding's
// tables and the library's buffer layout.
#include "mech_internal.h"

#include <cstdio>

int main() {
    for (int k = MECH_PAS; k <= MECH_CABUF; ++k) {
        const mech::KindShape s = mech::kind_shape(k);
        std::printf("%d %d %d %d %d %d\n", k, s.n_state, s.n_param, s.param_double, s.has_ica, s.has_gid);
    }
    return 0;
}
