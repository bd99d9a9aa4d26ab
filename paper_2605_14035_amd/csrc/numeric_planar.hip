// Numeric phase of planar domains (triangles in the plane): the kernels of numeric_impl.hpp instantiated
// for orders 1 to 4 (one translation unit per element family, built in parallel).
#include "numeric_impl.hpp"

namespace lfem {

void numeric_planar(Mesh &m, Pattern &p, const NumericOut &no, int variant, hipStream_t s)
{
    const Outs o = arrange(no);
    switch (m.etype) {
    case B2P1: run_type<ET<0, 2, 1>>(m, p, o, variant, s); break;
    case B2P2: run_type<ET<0, 2, 2>>(m, p, o, variant, s); break;
    case B2P3: run_type<ET<0, 2, 3>>(m, p, o, variant, s); break;
    case B2P4: run_type<ET<0, 2, 4>>(m, p, o, variant, s); break;
    default: throw Error{LFEM_EUNSUPPORTED, "element type"};
    }
}

}  // namespace lfem
