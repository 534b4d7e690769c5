// gfx950 kernels of the permutation-avoiding convolution.
//
// pass_kernel: one HBM pass = load an L x W tile into LDS (coalesced along
// whichever of the two tile dimensions is contiguous in memory), apply the
// pass's ops (grouped DIF / DIT stages and the fused product with the
// digit-reversed spectrum), store the tile back.  Every transform of the
// library -- a whole 1-D transform in LDS, the contiguous and the strided
// axis passes of 2-D/3-D grids, the fused middle pass, and the outer and
// inner halves of 1-D transforms too long for LDS -- is an instance of this
// kernel with a different descriptor (see pafc_internal.h).
//
// Stage order and arithmetic follow the paper's kernels: forward =
// A^T = product of B_{r,k}^T, block size k decreasing (Alg.
// alg:transposed-butterfly-kernel); inverse = conj(A) = product of
// conj(B_{r,k}), k increasing (Alg. alg:butterfly-related-kernel); with the
// mixed-radix stage sequence of Sec. "Mixed-radix framework".  Consecutive
// stages of equal radix are grouped into one register-resident R-point DFT
// plus one twiddle per element, which is the same linear map.
#include <hip/hip_runtime.h>

#include "pass_engine.h"

#include <algorithm>

namespace pafc {

template <typename T, int CLS>
__global__ void __launch_bounds__(class_max_threads<CLS>()) pass_kernel(const PassArgs* __restrict__ desc,
                                                   const void* in, void* out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  do_tile<T, CLS>(*desc, in, out, blockIdx.x, 0, lds);
}

// Batched form: block b processes work item tiles[first + b]; the pass
// descriptors of all size classes sit in device memory.
template <typename T, int CLS>
__global__ void __launch_bounds__(class_max_threads<CLS>()) batch_kernel(const PassArgs* __restrict__ descs,
                                                    const BatchTile* __restrict__ tiles,
                                                    uint32_t first, const void* in, void* out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const BatchTile bt = tiles[first + blockIdx.x];
  do_tile<T, CLS>(descs[bt.desc], in, out, bt.tile, bt.offset, lds);
}

// Persistent batched form: one launch for the whole batch.  A resident
// block claims whole problems from a device counter, in the host's order
// (largest first), and runs every pass of a problem itself, tile by tile;
// so a pass's dependence on the previous pass of the same problem is
// ordered by the block's own barriers, and blocks never wait for each
// other.  The last block to leave resets the control words, so the launch
// can be replayed (a captured graph) without a memset between launches.
template <typename T>
__global__ void __launch_bounds__(256) batch_persist_kernel(const PassArgs* __restrict__ descs,
                                                            const BatchJob* __restrict__ jobs,
                                                            uint32_t njobs, BatchCtl* ctl,
                                                            const void* in, void* out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  __shared__ uint32_t s_job;
  for (;;) {
    if (threadIdx.x == 0)
      s_job = __hip_atomic_fetch_add(&ctl->next, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint32_t k = __builtin_amdgcn_readfirstlane(s_job);
    __syncthreads();  // every thread has read s_job before thread 0 writes it again
    if (k >= njobs) break;
    const BatchJob j = jobs[k];
    for (uint32_t q = 0; q < j.npass; ++q) {
      const PassArgs& a = descs[j.desc + q];
      // the first pass reads the input, the later ones work in place on the
      // output (which the previous pass of this block wrote)
      const void* src = q == 0 ? in : out;
      for (uint32_t t = 0; t < a.ntiles; ++t) {
        do_tile<T, 0>(a, src, out, t, j.offset, lds);
        // LDS is reused by the next tile, and the next pass reads what this
        // one wrote to global memory: a workgroup-scope fence and barrier
        __syncthreads();
      }
    }
  }
  if (threadIdx.x == 0) {
    const uint32_t before =
        __hip_atomic_fetch_add(&ctl->exited, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (before == gridDim.x - 1) {  // every other block has left the loop
      __hip_atomic_store(&ctl->next, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctl->exited, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ------------------------------------------------------------ elementwise

template <typename T>
__global__ void scale_kernel(cx<T>* __restrict__ p, int64_t n, T s) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    cx<T> v = p[i];
    p[i] = {v.re * s, v.im * s};
  }
}

// Plain streaming copy (counter calibration).
__global__ void stream_copy_kernel(const double2* __restrict__ a, double2* __restrict__ b,
                                   int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// The same copy with 8 bytes per lane.
__global__ void stream_copy8_kernel(const uint64_t* __restrict__ a, uint64_t* __restrict__ b,
                                    int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// Streaming probes with the access pattern of a strided middle pass: the
// array is 256 rows of `cols` 16-byte elements, a tile is all 256 rows x 16
// columns (256-byte row segments), and each block walks the tiles
// blockIdx.x, + gridDim.x, ...  Per tile every thread moves 16 elements, all
// loads issued before the stores.  MUL: the output is x * h, h read
// contiguously in tile order (as a tile-major spectrum).
template <bool MUL>
__global__ void __launch_bounds__(256) tile_stream_kernel(const double2* __restrict__ x,
                                                          const double2* __restrict__ h,
                                                          double2* __restrict__ y,
                                                          uint32_t cols) {
  const uint32_t ntiles = cols / 16u;
  const uint32_t tid = threadIdx.x;
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    double2 v[16], w[16];
#pragma unroll
    for (uint32_t k = 0; k < 16; ++k) {
      const uint32_t idx = k * 256u + tid;  // row idx / 16, column idx % 16
      v[k] = x[(size_t)(idx >> 4) * cols + t * 16u + (idx & 15u)];
      if (MUL) w[k] = h[(size_t)t * 4096u + idx];
    }
#pragma unroll
    for (uint32_t k = 0; k < 16; ++k) {
      const uint32_t idx = k * 256u + tid;
      double2 o = v[k];
      if (MUL) o = double2{v[k].x * w[k].x - v[k].y * w[k].y, v[k].x * w[k].y + v[k].y * w[k].x};
      y[(size_t)(idx >> 4) * cols + t * 16u + (idx & 15u)] = o;
    }
  }
}

// Read-only sweep: every 16-byte element read once; one 16-byte sum per
// block is written (so the reads cannot be dropped), a negligible write.
__global__ void __launch_bounds__(256) stream_read_kernel(const double2* __restrict__ a,
                                                          double2* __restrict__ out, int64_t n) {
  __shared__ double2 part[256];
  double2 acc = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = a[i];
    acc.x += v.x;
    acc.y += v.y;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (uint32_t h = blockDim.x / 2; h > 0; h /= 2) {
    if (threadIdx.x < h) {
      part[threadIdx.x].x += part[threadIdx.x + h].x;
      part[threadIdx.x].y += part[threadIdx.x + h].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = part[0];
}

template <typename T>
__global__ void mul_kernel(const cx<T>* __restrict__ x, const cx<T>* __restrict__ h,
                           cx<T>* __restrict__ y, int64_t n, T s, uint32_t nt_h) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = cscale(cmul(x[i], nt_h ? ld_nt(h + i) : h[i]), s);
}

// Per-axis index-reversal permutation as one HBM pass (the explicit variant's
// Alg. alg:index-reversal-permutation), with an optional product:
//   out[k_1..k_d] = in[map_1[k_1], ..., map_d[k_d]] (* h[k_1..k_d] * s).
// One block handles `rows` output rows of the last axis; a source row is
// staged through LDS so that both the global read and the global write are
// contiguous; the within-row reversal happens on the LDS read.
template <typename T>
__global__ void __launch_bounds__(256) permute_rows_kernel(
    const cx<T>* __restrict__ in, cx<T>* __restrict__ out, const cx<T>* __restrict__ h,
    const int32_t* __restrict__ map0, const int32_t* __restrict__ map1,
    const int32_t* __restrict__ map_last, uint32_t n0, uint32_t n1, uint32_t nlast,
    uint32_t rows_per_block, uint32_t nrows, T s, uint32_t nt_h) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const uint32_t row0 = blockIdx.x * rows_per_block;
  const uint32_t nr = min(rows_per_block, nrows - row0);
  const uint32_t tot = nr * nlast;
  for (uint32_t x = threadIdx.x; x < tot; x += blockDim.x) {
    const uint32_t rr = x / nlast, k = x - rr * nlast;
    const uint32_t row = row0 + rr;
    const uint32_t k0 = row / n1, k1 = row - k0 * n1;
    const uint32_t srow = (n0 > 1 ? (uint32_t)map0[k0] : 0u) * n1 + (n1 > 1 ? (uint32_t)map1[k1] : 0u);
    lds[lds_phys(x)] = in[(int64_t)srow * nlast + k];
  }
  __syncthreads();
  for (uint32_t x = threadIdx.x; x < tot; x += blockDim.x) {
    const uint32_t rr = x / nlast, k = x - rr * nlast;
    const int64_t o = (int64_t)(row0 + rr) * nlast + k;
    cx<T> v = lds[lds_phys(rr * nlast + (uint32_t)map_last[k])];
    if (h) v = cscale(cmul(v, nt_h ? ld_nt(h + o) : h[o]), s);
    out[o] = v;
  }
}

// One-tile-per-block form: 4096 / NL whole output rows per block (NL a power
// of two), index maps staged in LDS, every source row load issued before the
// first store so that many blocks per CU keep loads in flight as in a copy.
template <typename T>
__global__ void __launch_bounds__(256) permute_tile_kernel(
    const cx<T>* __restrict__ in, cx<T>* __restrict__ out, const cx<T>* __restrict__ h,
    const int32_t* __restrict__ map0, const int32_t* __restrict__ map1,
    const int32_t* __restrict__ map_last, uint32_t n0, uint32_t n1, uint32_t log_nl,
    FastDiv div_n1, T s, uint32_t nt_h) {
  constexpr int EPT = 16;
  constexpr uint32_t TILE = 256 * EPT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  int32_t* lmap = reinterpret_cast<int32_t*>(lds + TILE + (TILE >> 4) + 2);
  const uint32_t nl = 1u << log_nl;
  const uint32_t rows_per_tile = TILE >> log_nl;
  int32_t* lsrc = lmap + nl;  // source row of each output row of the tile
  const uint32_t tid = threadIdx.x;
  const uint32_t row0 = blockIdx.x * rows_per_tile;
  for (uint32_t k = tid; k < nl; k += 256) lmap[k] = map_last[k];
  for (uint32_t r = tid; r < rows_per_tile; r += 256) {
    const uint32_t row = row0 + r;
    const uint32_t k0 = fdiv(row, div_n1), k1 = row - k0 * n1;
    lsrc[r] = (int32_t)((n0 > 1 ? (uint32_t)map0[k0] : 0u) * n1 + (n1 > 1 ? (uint32_t)map1[k1] : 0u));
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * TILE;
  cx<T> v[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const uint32_t x = tid + 256u * q;
    v[q] = in[((int64_t)lsrc[x >> log_nl] << log_nl) + (x & (nl - 1u))];
  }
#pragma unroll
  for (int q = 0; q < EPT; ++q) lds[lds_phys(tid + 256u * q)] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const uint32_t x = tid + 256u * q;
    const uint32_t rr = x >> log_nl, k = x & (nl - 1u);
    cx<T> w = lds[lds_phys((rr << log_nl) + (uint32_t)lmap[k])];
    if (h) w = cscale(cmul(w, nt_h ? ld_nt(h + base + x) : h[base + x]), s);
    out[base + x] = w;
  }
}

// Generic gather for axes too long for an LDS row:
//   out[o] = in[src(o)] (* h[o]), src from per-axis maps.
template <typename T>
__global__ void permute_gather_kernel(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                      const cx<T>* __restrict__ h,
                                      const int32_t* __restrict__ m0, const int32_t* __restrict__ m1,
                                      const int32_t* __restrict__ m2, uint32_t n0, uint32_t n1,
                                      uint32_t n2, int64_t n, T sc, uint32_t nt_h) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n;
       o += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k2 = (uint32_t)(o % n2);
    const int64_t q = o / n2;
    const uint32_t k1 = (uint32_t)(q % n1);
    const uint32_t k0 = (uint32_t)(q / n1);
    const int64_t s = ((int64_t)(n0 > 1 ? m0[k0] : 0) * n1 + (n1 > 1 ? m1[k1] : 0)) * n2 + m2[k2];
    cx<T> v = in[s];
    if (h) v = cscale(cmul(v, nt_h ? ld_nt(h + o) : h[o]), sc);
    out[o] = v;
  }
}

// A diagonal operator's spectrum written in the plan's layout: at position
// (p_0, p_1, p_2) the natural frequency of axis i is k_i = map_i[p_i] (or
// p_i when map_i is NULL; k_i < n_i), and the value combines the per-axis
// entries g[off_i + k_i]: mode 0 -> -1 / (sum of their real parts), 0 where the sum
// is 0; mode 1 -> the complex product.  Computed in FP64, rounded once.
template <typename T>
__global__ void symbol_kernel(cx<T>* __restrict__ H, const double2* __restrict__ g,
                              const int32_t* __restrict__ m0, const int32_t* __restrict__ m1,
                              const int32_t* __restrict__ m2, uint32_t n0, uint32_t n1,
                              uint32_t n2, uint32_t off0, uint32_t off1, uint32_t off2, int mode,
                              int64_t n) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n;
       o += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p2 = (uint32_t)(o % n2);
    const int64_t q = o / n2;
    const uint32_t p1 = (uint32_t)(q % n1);
    const uint32_t p0 = (uint32_t)(q / n1);
    const double2 a = g[off0 + (m0 ? m0[p0] : p0)];
    const double2 b = g[off1 + (m1 ? m1[p1] : p1)];
    const double2 c = g[off2 + (m2 ? m2[p2] : p2)];
    double re, im;
    if (mode == 0) {
      const double s = a.x + b.x + c.x;
      re = s == 0.0 ? 0.0 : -1.0 / s;
      im = 0.0;
    } else {
      const double abr = a.x * b.x - a.y * b.y, abi = a.x * b.y + a.y * b.x;
      re = abr * c.x - abi * c.y;
      im = abr * c.y + abi * c.x;
    }
    H[o] = cx<T>{(T)re, (T)im};
  }
}

// Index maps of the prime-factor route (Sec. "Prime factor framework"): a
// 1-D array of length n = N0 N1 N2 (pairwise coprime factors) and the
// N0 x N1 x N2 grid it is reindexed to.
//   gather:  out[(j0 N1 + j1) N2 + j2] = in[(t0[j0] + t1[j1] + t2[j2]) mod n]
//            (t_q[j] = j e_q mod n; with e_q = n / N_q this is the output
//            map of a filter's spectrum)
// n < 2^31; every table entry is below n.
template <typename T>
__global__ void pfa_gather_kernel(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                  const uint32_t* __restrict__ t0, const uint32_t* __restrict__ t1,
                                  const uint32_t* __restrict__ t2, FastDiv d1, FastDiv d2,
                                  uint32_t n) {
  for (uint32_t o = blockIdx.x * blockDim.x + threadIdx.x; o < n; o += gridDim.x * blockDim.x) {
    const uint32_t q = fdiv(o, d2);
    const uint32_t j2 = o - q * d2.d;
    const uint32_t j0 = fdiv(q, d1);
    const uint32_t j1 = q - j0 * d1.d;
    uint64_t s = (uint64_t)t0[j0] + t1[j1] + t2[j2];
    if (s >= n) s -= n;
    if (s >= n) s -= n;
    out[o] = in[s];
  }
}

// The CRT map itself, j <-> grid position ((j mod N0) N1 + j mod N1) N2 +
// j mod N2, in both directions (dir 0: grid[pos(j)] = in[j], the input map;
// dir 1: out[j] = grid[pos(j)], its inverse).  Element by element, one side
// of the map is read or written with a stride of about N1 N2 elements, one
// cache line per element.  Tiled instead: with U = N0 N1, each j is the pair
// (u, w) = (j mod U, j mod N2) and u + U k (k = (w - u) U^-1 mod N2) back.
// Tile (u0, w0) holds the pairs u = u0 + a, w = (w0 + b + a) mod N2 for
// a, b < 16: along a both u and w step by one, so j steps by one (16
// consecutive j); along b only w steps, 16 consecutive grid positions (up to
// a wrap of w).  The tiles u0, w0 in 16 Z cover every pair once (u < U,
// w0 + b < N2), and each passes through LDS, so both sides move runs of 16
// elements.  256 threads per tile; uinv = U^-1 mod N2.
template <typename T, int DIR>
__global__ void __launch_bounds__(256)
pfa_map_kernel(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, FastDiv d0, FastDiv d1,
               FastDiv d2, uint32_t U, uint32_t uinv, FastDiv dtw) {
  __shared__ cx<T> tile[16][17];
  const uint32_t tu = fdiv(blockIdx.x, dtw);
  const uint32_t u0 = tu * 16, w0 = (blockIdx.x - tu * dtw.d) * 16;
  const uint32_t N2 = d2.d;
  // element (a, b): false outside the tile's part of the index space
  auto locate = [&](uint32_t a, uint32_t b, uint32_t* j, uint32_t* g) -> bool {
    const uint32_t u = u0 + a, wb = w0 + b;
    if (u >= U || wb >= N2) return false;
    const uint32_t w = (wb + a) - fdiv(wb + a, d2) * N2;
    const uint32_t r0 = u - fdiv(u, d0) * d0.d;
    const uint32_t r1 = u - fdiv(u, d1) * d1.d;
    *g = (r0 * d1.d + r1) * N2 + w;
    const uint32_t um = u - fdiv(u, d2) * N2;
    const uint32_t dw = w >= um ? w - um : w + N2 - um;
    *j = u + U * (uint32_t)(((uint64_t)dw * uinv) % N2);
    return true;
  };
  const uint32_t hi = threadIdx.x >> 4, lo = threadIdx.x & 15u;
  uint32_t j, g;
  // read along the contiguous side of the source: j for dir 0, grid for 1
  const uint32_t ra = DIR == 0 ? lo : hi, rb = DIR == 0 ? hi : lo;
  if (locate(ra, rb, &j, &g)) tile[ra][rb] = in[DIR == 0 ? j : g];
  __syncthreads();
  const uint32_t wa = DIR == 0 ? hi : lo, wb = DIR == 0 ? lo : hi;
  if (locate(wa, wb, &j, &g)) out[DIR == 0 ? g : j] = tile[wa][wb];
}

// Bluestein's method (Sec. "Rader's and Bluestein's frameworks"): the
// length-n DFT as a length-m circular convolution (m >= 2n - 1) with the
// chirp c_j = w_{2n}^{j^2}:  DFT(x)_k = c_k [ (x o c, padded) (*) g ]_k, with
// g the filter of the inner plan (conj(c) on offsets |d| < n).  The inverse
// DFT reuses the same convolution through conjugation.
//   in:   a_j = x_j c_j (j < n), 0 (n <= j < m)
//   spec: Hn_k = c_k b_k (k < n)                 (a filter's spectrum)
//   mid:  b_k = conj(c_k b_k Hn_k) c_k (k < n), 0 (k >= n)
//   out:  y_j = conj(c_j b_j) s
template <typename T>
__global__ void blue_in_kernel(const cx<T>* __restrict__ x, const cx<T>* __restrict__ c,
                               cx<T>* __restrict__ a, int64_t n, int64_t m) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m;
       j += (int64_t)gridDim.x * blockDim.x)
    a[j] = j < n ? cmul(x[j], c[j]) : cx<T>{(T)0, (T)0};
}

template <typename T>
__global__ void blue_spec_kernel(const cx<T>* __restrict__ b, const cx<T>* __restrict__ c,
                                 cx<T>* __restrict__ hn, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    hn[k] = cmul(c[k], b[k]);
}

template <typename T>
__global__ void blue_mid_kernel(cx<T>* __restrict__ b, const cx<T>* __restrict__ c,
                                const cx<T>* __restrict__ hn, int64_t n, int64_t m) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m;
       k += (int64_t)gridDim.x * blockDim.x) {
    cx<T> v = {(T)0, (T)0};
    if (k < n) {
      const cx<T> z = cmul(cmul(c[k], b[k]), hn[k]);
      v = cmul(cx<T>{z.re, -z.im}, c[k]);
    }
    b[k] = v;
  }
}

template <typename T>
__global__ void blue_out_kernel(const cx<T>* __restrict__ b, const cx<T>* __restrict__ c,
                                cx<T>* __restrict__ y, int64_t n, T s) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const cx<T> z = cmul(c[j], b[j]);
    y[j] = cx<T>{z.re * s, -z.im * s};
  }
}


// Rader's algorithm (Sec. "Rader's and Bluestein's frameworks") for a prime
// length p with a generator g of the multiplicative group mod p, P1 = p - 1.
// With a_m = x[g^m] and the inner filter b_l = w_p^{g^{-l}}, the DFT at the
// nonzero frequencies is X[g^{-q}] = x_0 + (a (*) b)_q, a length-P1 circular
// convolution; X_0 = x_0 - sum_q (a (*) b)_q since sum_l b_l = -1.  The
// spectrum is kept in this q order (Hq[q] = H[g^{-q}], Hq[P1] = H_0), so the
// product needs no reordering, and the inverse DFT is the same convolution
// through conjugation: with w_m = conj(Y[g^m]) = conj(Yq[-m]),
// y[g^{-r}] = (Y_0 + conj((w (*) b)_r)) / p and y_0 = (Y_0 + sum_q Yq[q]) / p.
// Tables: pw[m] = g^m mod p (m < P1); lg[j] = -log_g(j) mod P1 (0 < j < p).
//   in:   a_m = x[pw[m]]
//   sums: mode 0 (filter): hq[q] = x_0 + u_q, block sums of u
//         mode 1 (product): u <- w in place, pairs (m, P1 - m) per thread,
//         block sums of u and of Yq
//   fin:  mode 0: hq[P1] = x_0 - sum u;  mode 1: consts = {Y_0, Y_0 + sum Yq}
//   out:  y_0 = s consts[1], y_j = s (consts[0] + conj(v[lg[j]]))
//   nat:  hq[q] = hn[pw[-q mod P1]], hq[P1] = hn[0]   (natural-order spectrum)
// Block sums are double, four per block (sum u re/im, sum Yq re/im), added
// in a fixed order, so results do not depend on scheduling.
template <typename T>
__global__ void rader_in_kernel(const cx<T>* __restrict__ x, const uint32_t* __restrict__ pw,
                                cx<T>* __restrict__ a, uint32_t P1) {
  for (uint32_t m = blockIdx.x * blockDim.x + threadIdx.x; m < P1; m += gridDim.x * blockDim.x)
    a[m] = x[pw[m]];
}

__device__ inline void block_sum4(double v[4], double* __restrict__ out) {
  __shared__ double red[4][256];
  for (int c = 0; c < 4; ++c) red[c][threadIdx.x] = v[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 4; ++c) out[c] = red[c][0];
}

template <typename T>
__global__ __launch_bounds__(256) void rader_sums_kernel(cx<T>* __restrict__ u,
                                                          const cx<T>* __restrict__ x,
                                                          cx<T>* __restrict__ hq,
                                                          double* __restrict__ part, uint32_t P1,
                                                          int mode) {
  const cx<T> x0 = x[0];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (mode == 0) {
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < P1; q += gridDim.x * blockDim.x) {
      const cx<T> v = u[q];
      acc[0] += (double)v.re;
      acc[1] += (double)v.im;
      hq[q] = cx<T>{x0.re + v.re, x0.im + v.im};
    }
  } else {
    const uint32_t half = P1 / 2;  // P1 is even
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t <= half;
         t += gridDim.x * blockDim.x) {
      const uint32_t tn = t == 0 ? 0 : P1 - t;
      const cx<T> ua = u[t], ub = u[tn];
      const cx<T> ya = cmul(cx<T>{x0.re + ua.re, x0.im + ua.im}, hq[t]);
      const cx<T> yb = cmul(cx<T>{x0.re + ub.re, x0.im + ub.im}, hq[tn]);
      u[t] = cx<T>{yb.re, -yb.im};
      acc[0] += (double)ua.re;
      acc[1] += (double)ua.im;
      acc[2] += (double)ya.re;
      acc[3] += (double)ya.im;
      if (tn != t) {
        u[tn] = cx<T>{ya.re, -ya.im};
        acc[0] += (double)ub.re;
        acc[1] += (double)ub.im;
        acc[2] += (double)yb.re;
        acc[3] += (double)yb.im;
      }
    }
  }
  block_sum4(acc, part + (size_t)blockIdx.x * 4);
}

template <typename T>
__global__ __launch_bounds__(256) void rader_fin_kernel(const double* __restrict__ part,
                                                         uint32_t nb, const cx<T>* __restrict__ x,
                                                         cx<T>* __restrict__ hq,
                                                         cx<T>* __restrict__ consts, uint32_t P1,
                                                         int mode) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x)
    for (int c = 0; c < 4; ++c) acc[c] += part[(size_t)b * 4 + c];
  __shared__ double tot[4];
  block_sum4(acc, tot);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double x0r = (double)x[0].re, x0i = (double)x[0].im;
  const double X0r = x0r - tot[0], X0i = x0i - tot[1];
  if (mode == 0) {
    hq[P1] = cx<T>{(T)X0r, (T)X0i};
    return;
  }
  const cx<T> h0 = hq[P1];
  const double Y0r = X0r * (double)h0.re - X0i * (double)h0.im;
  const double Y0i = X0r * (double)h0.im + X0i * (double)h0.re;
  consts[0] = cx<T>{(T)Y0r, (T)Y0i};
  consts[1] = cx<T>{(T)(Y0r + tot[2]), (T)(Y0i + tot[3])};
}

template <typename T>
__global__ void rader_out_kernel(const cx<T>* __restrict__ v, const uint32_t* __restrict__ lg,
                                 const cx<T>* __restrict__ consts, cx<T>* __restrict__ y,
                                 uint32_t p, T s) {
  const cx<T> y0 = consts[0];
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < p; j += gridDim.x * blockDim.x) {
    if (j == 0) {
      const cx<T> c1 = consts[1];
      y[0] = cx<T>{c1.re * s, c1.im * s};
    } else {
      const cx<T> w = v[lg[j]];
      y[j] = cx<T>{(y0.re + w.re) * s, (y0.im - w.im) * s};
    }
  }
}

template <typename T>
__global__ void rader_nat_kernel(const cx<T>* __restrict__ hn, const uint32_t* __restrict__ pw,
                                 cx<T>* __restrict__ hq, uint32_t P1) {
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q <= P1; q += gridDim.x * blockDim.x)
    hq[q] = q == P1 ? hn[0] : hn[pw[q == 0 ? 0 : P1 - q]];
}

}  // namespace pafc

// ----------------------------------------------------------------- launches

namespace pafc {

template <typename T>
static hipError_t set_lds_limit(const void* fn) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

template <typename T, int CLS>
static hipError_t launch_pass_t(const PassArgs* d_desc, uint32_t ntiles, const void* in,
                                void* out, uint32_t threads, size_t lds_bytes, hipStream_t s) {
  static bool init = false;
  if (!init) {
    hipError_t e = set_lds_limit<T>((const void*)pass_kernel<T, CLS>);
    if (e != hipSuccess) return e;
    init = true;
  }
  hipLaunchKernelGGL((pass_kernel<T, CLS>), dim3(ntiles), dim3(threads), lds_bytes, s, d_desc,
                     in, out);
  return hipGetLastError();
}

hipError_t launch_pass(bool dbl, int cls, const PassArgs* d_desc, uint32_t ntiles, const void* in,
                       void* out, uint32_t threads, size_t lds_bytes, hipStream_t s) {
  if (cls < 0 || cls > 2 || threads > (cls == 2 ? 1024u : 256u)) return hipErrorInvalidValue;
#define PAFC_LP(TT, CC) launch_pass_t<TT, CC>(d_desc, ntiles, in, out, threads, lds_bytes, s)
  if (dbl) return cls == 0 ? PAFC_LP(double, 0) : cls == 1 ? PAFC_LP(double, 1) : PAFC_LP(double, 2);
  return cls == 0 ? PAFC_LP(float, 0) : cls == 1 ? PAFC_LP(float, 1) : PAFC_LP(float, 2);
#undef PAFC_LP
}

template <typename T, int CLS>
static hipError_t launch_batch_t(const PassArgs* descs, const BatchTile* tiles, uint32_t first,
                                 uint32_t count, const void* in, void* out, uint32_t threads,
                                 size_t lds_bytes, hipStream_t s) {
  static bool init = false;
  if (!init) {
    hipError_t e = set_lds_limit<T>((const void*)batch_kernel<T, CLS>);
    if (e != hipSuccess) return e;
    init = true;
  }
  hipLaunchKernelGGL((batch_kernel<T, CLS>), dim3(count), dim3(threads), lds_bytes, s, descs,
                     tiles, first, in, out);
  return hipGetLastError();
}

hipError_t launch_batch(bool dbl, int cls, const PassArgs* descs, const BatchTile* tiles,
                        uint32_t first, uint32_t count, const void* in, void* out,
                        uint32_t threads, size_t lds_bytes, hipStream_t s) {
  if (count == 0) return hipSuccess;
  if (cls < 0 || cls > 2 || threads > (cls == 2 ? 1024u : 256u)) return hipErrorInvalidValue;
#define PAFC_LB(TT, CC) \
  launch_batch_t<TT, CC>(descs, tiles, first, count, in, out, threads, lds_bytes, s)
  if (dbl) return cls == 0 ? PAFC_LB(double, 0) : cls == 1 ? PAFC_LB(double, 1) : PAFC_LB(double, 2);
  return cls == 0 ? PAFC_LB(float, 0) : cls == 1 ? PAFC_LB(float, 1) : PAFC_LB(float, 2);
#undef PAFC_LB
}

template <typename T>
static const void* persist_fn() {
  return (const void*)batch_persist_kernel<T>;
}

int batch_persist_blocks_per_cu(bool dbl, size_t lds_bytes) {
  const void* fn = dbl ? persist_fn<double>() : persist_fn<float>();
  // the kernel's static LDS (the claimed job) counts against the same 160 KB
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 159 * 1024) != hipSuccess)
    return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, lds_bytes) != hipSuccess) return 0;
  return nb;
}

// The dynamic LDS limit was raised at planning (batch_persist_blocks_per_cu).
hipError_t launch_batch_persist(bool dbl, const PassArgs* descs, const BatchJob* jobs,
                                uint32_t njobs, BatchCtl* ctl, uint32_t grid, size_t lds_bytes,
                                const void* in, void* out, hipStream_t s) {
  if (grid == 0) return hipErrorInvalidValue;
  if (dbl)
    hipLaunchKernelGGL(batch_persist_kernel<double>, dim3(grid), dim3(256), lds_bytes, s, descs,
                       jobs, njobs, ctl, in, out);
  else
    hipLaunchKernelGGL(batch_persist_kernel<float>, dim3(grid), dim3(256), lds_bytes, s, descs,
                       jobs, njobs, ctl, in, out);
  return hipGetLastError();
}

static uint32_t grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (uint32_t)b;
}

hipError_t launch_scale(bool dbl, void* p, int64_t n, double s, hipStream_t st) {
  if (dbl)
    hipLaunchKernelGGL(scale_kernel<double>, dim3(grid_for(n)), dim3(256), 0, st,
                       (cx<double>*)p, n, s);
  else
    hipLaunchKernelGGL(scale_kernel<float>, dim3(grid_for(n)), dim3(256), 0, st,
                       (cx<float>*)p, n, (float)s);
  return hipGetLastError();
}

hipError_t launch_symbol(bool dbl, void* H, const void* g, const int32_t* m0, const int32_t* m1,
                         const int32_t* m2, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t off0,
                         uint32_t off1, uint32_t off2, int mode, hipStream_t st) {
  const int64_t n = (int64_t)n0 * n1 * n2;
  if (dbl)
    hipLaunchKernelGGL(symbol_kernel<double>, dim3(grid_for(n)), dim3(256), 0, st,
                       (cx<double>*)H, (const double2*)g, m0, m1, m2, n0, n1, n2, off0, off1,
                       off2, mode, n);
  else
    hipLaunchKernelGGL(symbol_kernel<float>, dim3(grid_for(n)), dim3(256), 0, st,
                       (cx<float>*)H, (const double2*)g, m0, m1, m2, n0, n1, n2, off0, off1,
                       off2, mode, n);
  return hipGetLastError();
}

hipError_t launch_pfa_gather(bool dbl, const void* in, void* out, const uint32_t* t0,
                             const uint32_t* t1, const uint32_t* t2, uint32_t N1, uint32_t N2,
                             uint32_t n, hipStream_t st) {
  const FastDiv d1 = make_fastdiv(N1), d2 = make_fastdiv(N2);
  if (dbl)
    hipLaunchKernelGGL(pfa_gather_kernel<double>, dim3(grid_for(n)), dim3(256), 0, st,
                       (const cx<double>*)in, (cx<double>*)out, t0, t1, t2, d1, d2, n);
  else
    hipLaunchKernelGGL(pfa_gather_kernel<float>, dim3(grid_for(n)), dim3(256), 0, st,
                       (const cx<float>*)in, (cx<float>*)out, t0, t1, t2, d1, d2, n);
  return hipGetLastError();
}

hipError_t launch_pfa_map(bool dbl, int dir, const void* in, void* out, uint32_t N0, uint32_t N1,
                          uint32_t N2, uint32_t uinv, hipStream_t st) {
  const FastDiv d0 = make_fastdiv(N0), d1 = make_fastdiv(N1), d2 = make_fastdiv(N2);
  const uint32_t U = N0 * N1;
  const uint32_t tw = (N2 + 15) / 16;
  const dim3 grid(((U + 15) / 16) * tw);
  const FastDiv dtw = make_fastdiv(tw);
#define PAFC_MAP_LAUNCH(T, D)                                                              \
  hipLaunchKernelGGL((pfa_map_kernel<T, D>), grid, dim3(256), 0, st, (const cx<T>*)in,   \
                     (cx<T>*)out, d0, d1, d2, U, uinv, dtw)
  if (dbl) {
    if (dir == 0) PAFC_MAP_LAUNCH(double, 0);
    else PAFC_MAP_LAUNCH(double, 1);
  } else {
    if (dir == 0) PAFC_MAP_LAUNCH(float, 0);
    else PAFC_MAP_LAUNCH(float, 1);
  }
#undef PAFC_MAP_LAUNCH
  return hipGetLastError();
}

// stage 0 in, 1 spec, 2 mid, 3 out (see blue_*_kernel)
hipError_t launch_bluestein(bool dbl, int stage, const void* src, const void* c, void* dst,
                            const void* hn, int64_t n, int64_t m, double s, hipStream_t st) {
  const uint32_t g = grid_for(stage == 0 || stage == 2 ? m : n);
#define PAFC_BL(TT)                                                                              \
  switch (stage) {                                                                               \
    case 0:                                                                                      \
      hipLaunchKernelGGL(blue_in_kernel<TT>, dim3(g), dim3(256), 0, st, (const cx<TT>*)src,      \
                         (const cx<TT>*)c, (cx<TT>*)dst, n, m);                                  \
      break;                                                                                     \
    case 1:                                                                                      \
      hipLaunchKernelGGL(blue_spec_kernel<TT>, dim3(g), dim3(256), 0, st, (const cx<TT>*)src,    \
                         (const cx<TT>*)c, (cx<TT>*)dst, n);                                     \
      break;                                                                                     \
    case 2:                                                                                      \
      hipLaunchKernelGGL(blue_mid_kernel<TT>, dim3(g), dim3(256), 0, st, (cx<TT>*)dst,           \
                         (const cx<TT>*)c, (const cx<TT>*)hn, n, m);                             \
      break;                                                                                     \
    case 3:                                                                                      \
      hipLaunchKernelGGL(blue_out_kernel<TT>, dim3(g), dim3(256), 0, st, (const cx<TT>*)src,     \
                         (const cx<TT>*)c, (cx<TT>*)dst, n, (TT)s);                              \
      break;                                                                                     \
    default:                                                                                     \
      return hipErrorInvalidValue;                                                               \
  }
  if (dbl) {
    PAFC_BL(double)
  } else {
    PAFC_BL(float)
  }
#undef PAFC_BL
  return hipGetLastError();
}

// stage 0 in, 1 sums (mode 0/1), 2 fin (mode 0/1), 3 out, 4 natural spectrum
// (see rader_*_kernel); the sums stage uses at most kRaderBlocks blocks.
hipError_t launch_rader(bool dbl, int stage, int mode, const void* src, const void* x, void* dst,
                        void* hq, const uint32_t* pw, const uint32_t* lg, double* part,
                        void* consts, uint32_t p, double s, hipStream_t st) {
  const uint32_t P1 = p - 1;
  uint32_t nb = (P1 / 2 + 1 + 255) / 256;
  if (nb > kRaderBlocks) nb = kRaderBlocks;
#define PAFC_RD(TT)                                                                              \
  switch (stage) {                                                                               \
    case 0:                                                                                      \
      hipLaunchKernelGGL(rader_in_kernel<TT>, dim3(grid_for(P1)), dim3(256), 0, st,              \
                         (const cx<TT>*)src, pw, (cx<TT>*)dst, P1);                              \
      break;                                                                                     \
    case 1:                                                                                      \
      hipLaunchKernelGGL(rader_sums_kernel<TT>, dim3(nb), dim3(256), 0, st, (cx<TT>*)dst,        \
                         (const cx<TT>*)x, (cx<TT>*)hq, part, P1, mode);                         \
      break;                                                                                     \
    case 2:                                                                                      \
      hipLaunchKernelGGL(rader_fin_kernel<TT>, dim3(1), dim3(256), 0, st, part, nb,              \
                         (const cx<TT>*)x, (cx<TT>*)hq, (cx<TT>*)consts, P1, mode);              \
      break;                                                                                     \
    case 3:                                                                                      \
      hipLaunchKernelGGL(rader_out_kernel<TT>, dim3(grid_for(p)), dim3(256), 0, st,              \
                         (const cx<TT>*)src, lg, (const cx<TT>*)consts, (cx<TT>*)dst, p, (TT)s); \
      break;                                                                                     \
    case 4:                                                                                      \
      hipLaunchKernelGGL(rader_nat_kernel<TT>, dim3(grid_for(p)), dim3(256), 0, st,              \
                         (const cx<TT>*)src, pw, (cx<TT>*)hq, P1);                               \
      break;                                                                                     \
    default:                                                                                     \
      return hipErrorInvalidValue;                                                               \
  }
  if (dbl) {
    PAFC_RD(double)
  } else {
    PAFC_RD(float)
  }
#undef PAFC_RD
  return hipGetLastError();
}

hipError_t launch_stream_copy(int kind, const void* src, void* dst, int64_t n16, hipStream_t st) {
  if (kind == 0)
    hipLaunchKernelGGL(stream_copy_kernel, dim3(grid_for(n16)), dim3(256), 0, st,
                       (const double2*)src, (double2*)dst, n16);
  else if (kind == 1)
    hipLaunchKernelGGL(stream_copy8_kernel, dim3(grid_for(2 * n16)), dim3(256), 0, st,
                       (const uint64_t*)src, (uint64_t*)dst, 2 * n16);
  else if (kind == 2)  // at most 65536 blocks, so at most 1 MiB of dst is written
    hipLaunchKernelGGL(stream_read_kernel, dim3(grid_for(n16)), dim3(256), 0, st,
                       (const double2*)src, (double2*)dst, n16);
  else if (kind == 3 || kind == 4) {  // n16 = 256 rows x cols, cols a multiple of 16
    const uint32_t cols = (uint32_t)(n16 / 256);
    const uint32_t grid = std::min<uint32_t>(cols / 16u, 512u);
    const double2* x = (const double2*)src;
    if (kind == 3)
      hipLaunchKernelGGL(tile_stream_kernel<false>, dim3(grid), dim3(256), 0, st, x, x,
                         (double2*)dst, cols);
    else
      hipLaunchKernelGGL(tile_stream_kernel<true>, dim3(grid), dim3(256), 0, st, x, x + n16,
                         (double2*)dst, cols);
  } else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_mul(bool dbl, const void* x, const void* h, void* y, int64_t n, double s,
                      bool nt_h, hipStream_t st) {
  if (dbl)
    hipLaunchKernelGGL(mul_kernel<double>, dim3(grid_for(n)), dim3(256), 0, st,
                       (const cx<double>*)x, (const cx<double>*)h, (cx<double>*)y, n, s,
                       (uint32_t)nt_h);
  else
    hipLaunchKernelGGL(mul_kernel<float>, dim3(grid_for(n)), dim3(256), 0, st,
                       (const cx<float>*)x, (const cx<float>*)h, (cx<float>*)y, n, (float)s,
                       (uint32_t)nt_h);
  return hipGetLastError();
}

hipError_t launch_permute_rows(bool dbl, const void* in, void* out, const void* h,
                               const int32_t* m0, const int32_t* m1, const int32_t* mlast,
                               uint32_t n0, uint32_t n1, uint32_t nlast, uint32_t rows_per_block,
                               double s, bool nt_h, hipStream_t st) {
  static bool init_d = false, init_f = false;
  const uint32_t nrows = n0 * n1;
  const uint32_t blocks = (nrows + rows_per_block - 1) / rows_per_block;
  const size_t elem = dbl ? 16 : 8;
  const uint32_t tot = rows_per_block * nlast;
  const size_t lds = (size_t)(tot + (tot >> 4) + 1) * elem;
  if (dbl) {
    if (!init_d) {
      hipError_t e = set_lds_limit<double>((const void*)permute_rows_kernel<double>);
      if (e != hipSuccess) return e;
      init_d = true;
    }
    hipLaunchKernelGGL(permute_rows_kernel<double>, dim3(blocks), dim3(256), lds, st,
                       (const cx<double>*)in, (cx<double>*)out, (const cx<double>*)h, m0, m1,
                       mlast, n0, n1, nlast, rows_per_block, nrows, s, (uint32_t)nt_h);
  } else {
    if (!init_f) {
      hipError_t e = set_lds_limit<float>((const void*)permute_rows_kernel<float>);
      if (e != hipSuccess) return e;
      init_f = true;
    }
    hipLaunchKernelGGL(permute_rows_kernel<float>, dim3(blocks), dim3(256), lds, st,
                       (const cx<float>*)in, (cx<float>*)out, (const cx<float>*)h, m0, m1, mlast,
                       n0, n1, nlast, rows_per_block, nrows, (float)s, (uint32_t)nt_h);
  }
  return hipGetLastError();
}

hipError_t launch_permute_tile(bool dbl, const void* in, void* out, const void* h,
                               const int32_t* m0, const int32_t* m1, const int32_t* mlast,
                               uint32_t n0, uint32_t n1, uint32_t log_nl, double s, bool nt_h,
                               hipStream_t st) {
  const uint32_t tile = 4096;
  const uint64_t total = (uint64_t)n0 * n1 << log_nl;
  if ((1u << log_nl) > tile || total % tile != 0) return hipErrorInvalidValue;
  const uint32_t ntiles = (uint32_t)(total / tile);
  const size_t elem = dbl ? 16 : 8;
  const size_t lds = (size_t)(tile + (tile >> 4) + 2) * elem + (((size_t)1 << log_nl) + (tile >> log_nl)) * 4;
  const void* fn = dbl ? (const void*)permute_tile_kernel<double> : (const void*)permute_tile_kernel<float>;
  static bool init[2] = {false, false};
  if (!init[dbl]) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    init[dbl] = true;
  }
  const FastDiv dn1 = make_fastdiv(n1);
  if (dbl)
    hipLaunchKernelGGL(permute_tile_kernel<double>, dim3(ntiles), dim3(256), lds, st,
                       (const cx<double>*)in, (cx<double>*)out, (const cx<double>*)h, m0, m1,
                       mlast, n0, n1, log_nl, dn1, s, (uint32_t)nt_h);
  else
    hipLaunchKernelGGL(permute_tile_kernel<float>, dim3(ntiles), dim3(256), lds, st,
                       (const cx<float>*)in, (cx<float>*)out, (const cx<float>*)h, m0, m1, mlast,
                       n0, n1, log_nl, dn1, (float)s, (uint32_t)nt_h);
  return hipGetLastError();
}

hipError_t launch_permute_gather(bool dbl, const void* in, void* out, const void* h,
                                 const int32_t* m0, const int32_t* m1, const int32_t* m2,
                                 uint32_t n0, uint32_t n1, uint32_t n2, double s, bool nt_h,
                                 hipStream_t st) {
  const int64_t n = (int64_t)n0 * n1 * n2;
  if (dbl)
    hipLaunchKernelGGL(permute_gather_kernel<double>, dim3(grid_for(n)), dim3(256), 0, st,
                       (const cx<double>*)in, (cx<double>*)out, (const cx<double>*)h, m0, m1, m2,
                       n0, n1, n2, n, s, (uint32_t)nt_h);
  else
    hipLaunchKernelGGL(permute_gather_kernel<float>, dim3(grid_for(n)), dim3(256), 0, st,
                       (const cx<float>*)in, (cx<float>*)out, (const cx<float>*)h, m0, m1, m2,
                       n0, n1, n2, n, (float)s, (uint32_t)nt_h);
  return hipGetLastError();
}

}  // namespace pafc
