// Forward instantiations of the dense sweep kernel (qp_fast_impl.h).
#include "qp_fast_impl.h"

QPF_INST(1, 1, false) QPF_INST(1, 2, false) QPF_INST(1, 3, false) QPF_INST(1, 4, false)
QPF_INST(2, 1, false) QPF_INST(2, 2, false) QPF_INST(2, 3, false) QPF_INST(2, 4, false)
QPF_INST(3, 1, false) QPF_INST(3, 2, false) QPF_INST(3, 3, false) QPF_INST(3, 4, false)
QPF_INST(4, 1, false) QPF_INST(4, 2, false) QPF_INST(4, 3, false) QPF_INST(4, 4, false)

size_t fast_lds_bytes(int n, int nvm, int ns, bool bwd, int rscap, int cscap)
{
    return qpfast::lds_bytes(n, nvm, ns, bwd, rscap, cscap);
}
