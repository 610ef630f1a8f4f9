// sweep_stream.hip -- dispatch of the z-march half-sweep by storage codec.
#include "kernels.h"

namespace hsg {

template <int STORE>
hipError_t launch_stream_s(const MultiStreamArgs &m, int kind, bool energy, int fuse, unsigned threads,
                           size_t lds_bytes, hipStream_t s);

hipError_t launch_half_sweep_stream(const MultiStreamArgs &m, int storage, int kind, bool energy, int fuse,
                                    unsigned threads, size_t lds_bytes, hipStream_t s)
{
    if (threads == 0 || threads > (unsigned)kBlock || m.n_groups < 1 || m.n_groups > kMaxStreamGroups)
        return hipErrorInvalidValue;
    switch (storage) {
    case 0: return launch_stream_s<0>(m, kind, energy, fuse, threads, lds_bytes, s);
    case 1: return launch_stream_s<1>(m, kind, energy, fuse, threads, lds_bytes, s);
    case 2: return launch_stream_s<2>(m, kind, energy, fuse, threads, lds_bytes, s);
    case 3: return launch_stream_s<3>(m, kind, energy, fuse, threads, lds_bytes, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hsg
