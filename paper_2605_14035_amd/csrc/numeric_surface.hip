// Numeric phase of surfaces (triangles in space): the kernels of numeric_impl.hpp instantiated
// for orders 1 to 4 (one translation unit per element family, built in parallel).
#include "numeric_impl.hpp"

namespace lfem {

void numeric_surface(Mesh &m, Pattern &p, const NumericOut &no, int variant, hipStream_t s)
{
    const Outs o = arrange(no);
    switch (m.etype) {
    case S2P1: run_type<ET<1, 2, 1>>(m, p, o, variant, s); break;
    case S2P2: run_type<ET<1, 2, 2>>(m, p, o, variant, s); break;
    case S2P3: run_type<ET<1, 2, 3>>(m, p, o, variant, s); break;
    case S2P4: run_type<ET<1, 2, 4>>(m, p, o, variant, s); break;
    default: throw Error{LFEM_EUNSUPPORTED, "element type"};
    }
}

}  // namespace lfem
