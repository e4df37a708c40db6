// Read-only streaming kernel: the HBM read rate a plain kernel reaches on this
// device, reported beside the vendor peak as the measured ceiling of the
// bandwidth-bound product kernels.  Every workgroup reads contiguous tiles of
// 256 x PU 16-byte vectors with non-temporal loads (the loads the coupling and
// near-field kernels issue), PU loads in flight per thread, grid-strided over the
// buffer; the loaded words are folded into one word that is stored only if it
// equals a constant no data here produces, so the loads stay live without a
// write stream.
#include <hip/hip_runtime.h>

#include "handle.h"

namespace h2 {
namespace {

constexpr int PT = 256;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int PU>
__global__ __launch_bounds__(PT) void stream_read(const u32x4* __restrict__ p, int64_t n16, uint32_t* __restrict__ sink) {
  constexpr int64_t tile = static_cast<int64_t>(PT) * PU;
  uint32_t acc = 0;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * tile; base < n16; base += static_cast<int64_t>(gridDim.x) * tile) {
    u32x4 v[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int64_t j = base + u * PT + threadIdx.x;
      v[u] = j < n16 ? __builtin_nontemporal_load(p + j) : u32x4{0, 0, 0, 0};
    }
#pragma unroll
    for (int u = 0; u < PU; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  if (acc == 0x9e3779b9u) sink[blockIdx.x] = acc;
}

template <int PU>
void launch_read(const void* data, int64_t n16, void* sink, int64_t sink_bytes, hipStream_t st) {
  const int64_t tile = static_cast<int64_t>(PT) * PU;
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((n16 + tile - 1) / tile, 4096));
  if (sink_bytes < grid * 4) throw Error(H2_EINVAL, "sink needs " + std::to_string(grid * 4) + " bytes");
  stream_read<PU><<<static_cast<unsigned>(grid), PT, 0, st>>>(static_cast<const u32x4*>(data), n16,
                                                             static_cast<uint32_t*>(sink));
  H2_HIP(hipGetLastError());
}

}  // namespace

void stream_read_launch(const void* data, int64_t bytes, int loads, void* sink, int64_t sink_bytes, hipStream_t st) {
  if (!data || !sink) throw Error(H2_EINVAL, "NULL pointer");
  if (bytes < 16 || bytes % 16 != 0) throw Error(H2_EINVAL, "bytes must be a positive multiple of 16");
  if (reinterpret_cast<uintptr_t>(data) % 16 != 0) throw Error(H2_EINVAL, "data must be 16-byte aligned");
  const int64_t n16 = bytes / 16;
  switch (loads) {
    case 4: launch_read<4>(data, n16, sink, sink_bytes, st); break;
    case 8: launch_read<8>(data, n16, sink, sink_bytes, st); break;
    case 16: launch_read<16>(data, n16, sink, sink_bytes, st); break;
    default: throw Error(H2_EINVAL, "loads in flight must be 4, 8 or 16");
  }
}

}  // namespace h2
