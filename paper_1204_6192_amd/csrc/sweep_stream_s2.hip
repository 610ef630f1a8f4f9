// Instantiation of the z-march kernels for spin storage codec 2 (one
// translation unit per codec so that the library builds in parallel).
#include "sweep_stream.h"

namespace hsg {
template hipError_t launch_stream_s<2>(const MultiStreamArgs &, int, bool, int, unsigned, size_t, hipStream_t);
}  // namespace hsg
