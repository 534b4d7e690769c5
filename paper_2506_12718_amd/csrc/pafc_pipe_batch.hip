// Launches of the pipelined pass kernel (pipe_kernel.h) over many problems
// of one length: the batched form's size classes, one launch per pass of a
// class, whose tiles run over every problem of the class through the
// problem table of PassArgs.
#include "pipe_kernel.h"

namespace pafc {

static const void* pipe_batch_lookup(bool dbl, int r, int g, int ng, int kind, int mode, int gm) {
  return pipe_lookup_t<true>(dbl, r, g, ng, kind, mode, gm, 0);
}

// Resident blocks per CU of a batched instance (0: no such instance, or an
// error).  Also raises the instance's dynamic LDS limit, before any launch.
int pipe_batch_blocks_per_cu(bool dbl, int r, int g, int ng, int kind, int mode,
                             uint32_t threads, size_t lds, int gm) {
  const void* fn = pipe_batch_lookup(dbl, r, g, ng, kind, mode, gm);
  if (!fn) return 0;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
    return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, (int)threads, lds) != hipSuccess) return 0;
  return nb;
}

hipError_t launch_pipe_batch(bool dbl, int r, int g, int ng, int kind, int mode, int gm,
                             const PassArgs* d, uint32_t grid, uint32_t threads, size_t lds,
                             const void* in, void* out, hipStream_t s) {
  const void* fn = pipe_batch_lookup(dbl, r, g, ng, kind, mode, gm);
  if (!fn) return hipErrorInvalidValue;
  void* args[] = {(void*)&d, (void*)&in, (void*)&out};
  return hipLaunchKernel(fn, dim3(grid), dim3(threads), args, lds, s);
}

}  // namespace pafc
