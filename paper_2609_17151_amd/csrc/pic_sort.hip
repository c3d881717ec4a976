// Stable sort of the particles of every segment of one species by cell.
#include "pic_internal.h"
#include "pic_kernels.h"

namespace pic {

hipError_t launch_sort(const DevPtrs&, int, int64_t, void*, size_t, hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace pic
