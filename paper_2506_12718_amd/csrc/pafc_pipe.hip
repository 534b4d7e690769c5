// Launches of the pipelined pass kernel (pipe_kernel.h) for single
// problems: one transform or convolution per launch.
#include <hip/hip_ext.h>

#include "pipe_kernel.h"

namespace pafc {

static const void* pipe_lookup(bool dbl, int r, int g, int ng, int kind, int mode, int gm = -1,
                               int xc = 0) {
  return pipe_lookup_t<false>(dbl, r, g, ng, kind, mode, gm < 0 ? g : gm, xc);
}

// A pass of the given kind with a shorter innermost group (gm < g) or
// folded length-2 column axes (xc > 0) in the given tile mode.
bool pipe_ext_supported(int r, int g, int ng, int gm, int xc, int kind, int mode) {
  return pipe_lookup(true, r, g, ng, kind, mode, gm, xc) != nullptr;
}

bool pipe_supported(int r, int g, int ng) {
  return pipe_lookup(true, r, g, ng, PIPE_FWD, MODE_CONTIG) != nullptr;
}

bool pipe_outer_supported(int r, int g, int ng) {
  return pipe_lookup(true, r, g, ng, PIPE_FWD, MODE_OUTER) != nullptr;
}

// Most threads a block of the pipelined kernel for groups r^g may have (xc:
// folded column axes of a middle pass).
int pipe_thread_limit(int r, int g, bool dbl, int xc) {
  if ((r == 3 || r == 5) && g == 1) return 1024;
  if (r == 3 && g == 2) return 512;  // radix-9 items: 2 waves per SIMD unspilled
  return xc > 0 && !dbl ? 512 : 256;
}

// Most threads a block of a uniform pipelined instance (no short group, no
// folded columns) may have: 512 for 4096-long axes in four radix-8 groups,
// as pipe_block_limit compiles them, else the radix's own limit.
int pipe_uniform_threads(int r, int g, int ng) {
  if (ipow(r, g) == 4 && ng == 6) return 1024;
  return ipow(r, g) == 8 && ng == 4 ? 512 : pipe_thread_limit(r, g, true, 0);
}

// Resident blocks per CU of a pipelined kernel instance (0 on error).
int pipe_blocks_per_cu(bool dbl, int r, int g, int ng, int kind, int mode, uint32_t threads,
                       size_t lds, int gm, int xc) {
  const void* fn = pipe_lookup(dbl, r, g, ng, kind, mode, gm, xc);
  if (!fn) return 0;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
    return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, (int)threads, lds) != hipSuccess) return 0;
  return nb;
}

hipError_t launch_pipe_htm(bool dbl, int r, int g, int ng, int mode, const PassArgs* d,
                           uint32_t ntiles, uint32_t threads, const void* src, void* dst,
                           hipStream_t s) {
  const uint32_t grid = ntiles < 8192u ? ntiles : 8192u;
#define PAFC_HTM_GO(rr, gg, nn)                                                               \
  if (r == rr && g == gg && ng == nn) {                                                       \
    if (dbl) {                                                                                \
      if (mode == MODE_CONTIG)                                                                \
        hipLaunchKernelGGL((pipe_htm_kernel<double, rr, gg, nn, MODE_CONTIG>), dim3(grid),    \
                           dim3(threads), 0, s, d, src, dst);                                 \
      else                                                                                    \
        hipLaunchKernelGGL((pipe_htm_kernel<double, rr, gg, nn, MODE_STRIDED>), dim3(grid),   \
                           dim3(threads), 0, s, d, src, dst);                                 \
    } else {                                                                                  \
      if (mode == MODE_CONTIG)                                                                \
        hipLaunchKernelGGL((pipe_htm_kernel<float, rr, gg, nn, MODE_CONTIG>), dim3(grid),     \
                           dim3(threads), 0, s, d, src, dst);                                 \
      else                                                                                    \
        hipLaunchKernelGGL((pipe_htm_kernel<float, rr, gg, nn, MODE_STRIDED>), dim3(grid),    \
                           dim3(threads), 0, s, d, src, dst);                                 \
    }                                                                                         \
    return hipGetLastError();                                                                 \
  }
  PAFC_PIPE_SHAPES(PAFC_HTM_GO)
#undef PAFC_HTM_GO
  return hipErrorInvalidValue;
}

hipError_t launch_pipe(bool dbl, int r, int g, int ng, int kind, int mode, const PassArgs* d,
                       uint32_t grid, uint32_t threads, size_t lds, const void* in, void* out,
                       hipStream_t s, int gm, int xc, hipEvent_t t0, hipEvent_t t1) {
  const void* fn = pipe_lookup(dbl, r, g, ng, kind, mode, gm, xc);
  if (!fn) return hipErrorInvalidValue;
  // the LDS limit of every instance is raised when its occupancy is queried
  // at plan time (pipe_blocks_per_cu), before any launch
  void* args[] = {(void*)&d, (void*)&in, (void*)&out};
  // Timing events, when given, take the dispatch's own start and end
  // timestamps: no marker packet enters the stream around the launch.
  if (t0 || t1) return hipExtLaunchKernel(fn, dim3(grid), dim3(threads), args, lds, s, t0, t1, 0);
  return hipLaunchKernel(fn, dim3(grid), dim3(threads), args, lds, s);
}

}  // namespace pafc
