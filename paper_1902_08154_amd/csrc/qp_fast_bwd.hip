// Adjoint instantiations of the dense sweep kernel (qp_fast_impl.h).
#include "qp_fast_impl.h"

QPF_INST(1, 1, true) QPF_INST(1, 2, true) QPF_INST(1, 3, true) QPF_INST(1, 4, true)
QPF_INST(2, 1, true) QPF_INST(2, 2, true) QPF_INST(2, 3, true) QPF_INST(2, 4, true)
QPF_INST(3, 1, true) QPF_INST(3, 2, true) QPF_INST(3, 3, true) QPF_INST(3, 4, true)
QPF_INST(4, 1, true) QPF_INST(4, 2, true) QPF_INST(4, 3, true) QPF_INST(4, 4, true)
