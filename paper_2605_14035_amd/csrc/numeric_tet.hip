// Numeric phase of tetrahedral domains: the kernels of numeric_impl.hpp instantiated
// for orders 1 to 4 (one translation unit per element family, built in parallel).
#include "numeric_impl.hpp"

namespace lfem {

void numeric_tet(Mesh &m, Pattern &p, const NumericOut &no, int variant, hipStream_t s)
{
    const Outs o = arrange(no);
    switch (m.etype) {
    case B3P1: run_type<ET<0, 3, 1>>(m, p, o, variant, s); break;
    case B3P2: run_type<ET<0, 3, 2>>(m, p, o, variant, s); break;
    case B3P3: run_type<ET<0, 3, 3>>(m, p, o, variant, s); break;
    case B3P4: run_type<ET<0, 3, 4>>(m, p, o, variant, s); break;
    default: throw Error{LFEM_EUNSUPPORTED, "element type"};
    }
}

}  // namespace lfem
