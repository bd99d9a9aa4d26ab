// Numeric phase of curves (segments in the plane): the kernels of numeric_impl.hpp instantiated
// for P1 and P2 (one translation unit per element family, built in parallel).
#include "numeric_impl.hpp"

namespace lfem {

void numeric_curve(Mesh &m, Pattern &p, const NumericOut &no, int variant, hipStream_t s)
{
    const Outs o = arrange(no);
    if (m.etype == S1P1) run_type<ET<1, 1, 1>>(m, p, o, variant, s);
    else run_type<ET<1, 1, 2>>(m, p, o, variant, s);
}

}  // namespace lfem
