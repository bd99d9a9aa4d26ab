// Numeric phase of tetrahedral domains: the kernels of numeric_impl.hpp instantiated
// for orders 1 and 2 (one translation unit per element family, built in parallel).
#include "numeric_impl.hpp"

namespace lfem {

void numeric_tet(Mesh &m, Pattern &p, const NumericOut &no, int variant, hipStream_t s)
{
    const Outs o = arrange(no);
    if (m.etype == B3P1) run_type<ET<0, 3, 1>>(m, p, o, variant, s);
    else run_type<ET<0, 3, 2>>(m, p, o, variant, s);
}

}  // namespace lfem
