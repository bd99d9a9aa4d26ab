// Batched multi-mesh assembly (placeholder until the persistent kernel lands).
#include "lfem_internal.hpp"

struct lfem_batch_s {
    int n = 0;
};

namespace lfem {

lfem_status batch_create(int, Mesh *const *, Pattern *const *, unsigned, int, hipStream_t,
                         lfem_batch_t *)
{
    throw Error{LFEM_EUNSUPPORTED, "batched assembly is not built yet"};
}

void batch_run(lfem_batch_t, double *const *, hipStream_t)
{
    throw Error{LFEM_EUNSUPPORTED, "batched assembly is not built yet"};
}

void batch_destroy(lfem_batch_t b) { delete b; }

}  // namespace lfem
