// The tile engine shared by the generic pass kernels (one tile per block, and
// batched): LDS twiddle tables, item geometry, the grouped
// DIF / DIT / MID ops, and the tile load / store loops.  See pafc_internal.h
// for the meaning of a pass, a tile and an op.
#pragma once

#include "kernel_common.h"

namespace pafc {

// Twiddle from the block's LDS copy of the two-level table.
template <typename T>
__device__ __forceinline__ cx<T> twiddle_lds(const PassArgs& a, const cx<T>* lds, uint32_t E) {
  const cx<T>* lo = lds + a.twl_off;
  const cx<T>* hi = lo + (1u << a.twl_bits);
  return cmul(lo[E & ((1u << a.twl_bits) - 1u)], hi[E >> a.twl_bits]);
}

// Stage the two-level twiddle table in LDS (from the flat or two-level
// global table); the caller synchronises before the first op.
template <typename T>
__device__ __forceinline__ void stage_twiddles(const PassArgs& a, cx<T>* lds) {
  if (a.twl_global) return;
  cx<T>* lo = lds + a.twl_off;
  cx<T>* hi = lo + (1u << a.twl_bits);
  const cx<T>* glo = reinterpret_cast<const cx<T>*>(a.tw_lo);
  const cx<T>* ghi = reinterpret_cast<const cx<T>*>(a.tw_hi);
  const uint32_t nlo = 1u << a.twl_bits;
  for (uint32_t e = threadIdx.x; e < nlo; e += blockDim.x) lo[e] = glo[e];
  for (uint32_t e = threadIdx.x; e < a.twl_nhi; e += blockDim.x)
    hi[e] = ghi ? ghi[e] : glo[e << a.twl_bits];
}

struct TileCtx {
  int64_t base;    // element offset of tile position (0, 0) in the data arrays
  int64_t off;     // packed offset of the problem (0 outside the batched form);
                   // the filter spectrum is per problem, so it is indexed
                   // without it
  uint32_t col0;   // global column of tile column 0
  uint32_t ls_i;   // LDS linear stride between positions
  uint32_t ls_c;   // LDS linear stride between columns
};

__device__ __forceinline__ TileCtx make_ctx(const PassArgs& a, uint32_t tile, int64_t off) {
  if (a.rev) tile = a.ntiles - 1u - tile;
  const uint32_t o = fdiv(tile, a.divTiles);
  const uint32_t cb = tile - o * a.tiles_per_slice;
  TileCtx t;
  t.col0 = cb * a.W;
  t.base = (int64_t)o * a.S_o + (int64_t)t.col0 * a.S_c + off;
  t.off = off;
  if (a.mode == MODE_STRIDED) {
    t.ls_i = a.W;
    t.ls_c = 1;
  } else {
    t.ls_i = 1;
    t.ls_c = a.L;
  }
  return t;
}

// Geometry of item `it` of an op: column c, block b, offset j < S.
struct OpItem {
  uint32_t c, j, gcol;
  bool valid;
  uint32_t lbase, lstep;   // LDS linear index of position i0 and step S
  int64_t gbase, gstep;    // global element index of position i0 and step S
};

__device__ __forceinline__ OpItem op_item(const PassArgs& a, const OpDesc& op, const TileCtx& t,
                                          uint32_t it) {
  if (op.cross) {  // legs along the columns of one tile row
    const uint32_t i = fdiv(it, op.divQ);
    const uint32_t q = it - i * op.divQ.d;
    const uint32_t hi = fdiv(q, op.divCs);
    const uint32_t lo = q - hi * op.divCs.d;
    OpItem m;
    m.c = 0;
    m.j = 0;
    m.gcol = t.col0;
    m.valid = true;
    m.lbase = i * t.ls_i + (hi * (uint32_t)op.R * op.cs + lo) * t.ls_c;
    m.lstep = op.cs * t.ls_c;
    m.gbase = 0;
    m.gstep = 0;
    return m;
  }
  const uint32_t S = op.S, K = op.K;
  uint32_t c, b, j;
  if (a.mode == MODE_STRIDED) {
    c = it & (a.W - 1u);
    const uint32_t rest = it >> a.logW;
    b = fdiv(rest, op.divS);
    j = rest - b * S;
  } else {
    const uint32_t q = fdiv(it, op.divS);
    j = it - q * S;
    c = fdiv(q, op.divNB);
    b = q - c * op.divNB.d;
  }
  OpItem m;
  m.c = c;
  m.j = j;
  m.gcol = t.col0 + c;
  m.valid = m.gcol < a.ncols;
  const uint32_t i0 = b * K + j;
  m.lbase = i0 * t.ls_i + c * t.ls_c;
  m.lstep = S * t.ls_i;
  m.gbase = t.base + (int64_t)i0 * a.S_i + (int64_t)c * a.S_c;
  m.gstep = (int64_t)S * a.S_i;
  return m;
}

// Global inputs of one item, in the order the op consumes them (DIF and MID
// read natural positions, DIT digit-reversed ones).
template <typename T, int r, int g, int TYPE, typename Dst>
__device__ __forceinline__ void fetch_item(const OpItem& m, const void* in,
                                           Dst& v) {
  constexpr int R = ipow(r, g);
  static_for<R>([&](auto s) {
    constexpr int p = TYPE == OP_DIT ? digrev<r, g>(s.value) : s.value;
    v[s.value] = m.valid ? ld_g<T>(in, m.gbase + p * m.gstep) : cx<T>{(T)0, (T)0};
  });
}

// One op over all items of the tile.  An op reads its R inputs from LDS or,
// when it is the first op of the pass and its access is coalesced
// (op.src_g), straight from global memory; symmetrically it writes to LDS or
// (op.dst_g, last op) straight to global memory.
template <typename T, int r, int g, int TYPE>
__device__ __forceinline__ void run_op(const PassArgs& a, const OpDesc& op, const TileCtx& t,
                                       cx<T>* lds, const void* in,
                                       void* out) {
  constexpr int R = ipow(r, g);
  for (uint32_t it = threadIdx.x; it < op.nitems; it += blockDim.x) {
    const OpItem m = op_item(a, op, t, it);
    auto put = [&](int k, cx<T> val) {
      if (op.dst_g) {
        if (m.valid) st_g<T>(out, m.gbase + k * m.gstep, val);
      } else {
        lds[lds_phys(m.lbase + k * m.lstep, a.lds_sh)] = val;
      }
    };
    cx<T> v[R];
    if (op.src_g) {
      fetch_item<T, r, g, TYPE>(m, in, v);
    } else {
      static_for<R>([&](auto s) {
        constexpr int p = TYPE == OP_DIT ? digrev<r, g>(s.value) : s.value;
        v[s.value] = lds[lds_phys(m.lbase + p * m.lstep, a.lds_sh)];
      });
    }
    if constexpr (TYPE == OP_DIF) {
      Dft<R, r, false, T>::run(v);
      if (op.tw) {
        const uint32_t jf = m.j * a.jmul + (a.col_in_j && m.valid ? fdiv(m.gcol, a.divJc) : 0u);
        if (a.twl_global) {
          // no LDS copy: one read of the global table per item, the other
          // twiddles as powers, w^(m jf) = (w^jf)^m (jf < Kf / R)
          const cx<T> w1 = twiddle<T>(a, jf * op.escale);
          cx<T> w = w1;
          static_for<R - 1>([&](auto mm) {
            v[mm.value + 1] = cmul(v[mm.value + 1], w);
            w = cmul(w, w1);
          });
        } else {
          uint32_t E = 0;
          static_for<R - 1>([&](auto mm) {
            E += jf;
            if (E >= op.Kf) E -= op.Kf;
            v[mm.value + 1] = cmul(v[mm.value + 1], twiddle_lds<T>(a, lds, E * op.escale));
          });
        }
      }
      static_for<R>([&](auto mm) { put(digrev<r, g>(mm.value), v[mm.value]); });
    } else if constexpr (TYPE == OP_DIT) {
      if (op.tw) {
        const uint32_t jf = m.j * a.jmul + (a.col_in_j && m.valid ? fdiv(m.gcol, a.divJc) : 0u);
        if (a.twl_global) {  // as in the DIF op
          const cx<T> w1 = twiddle<T>(a, jf * op.escale);
          cx<T> w = w1;
          static_for<R - 1>([&](auto mm) {
            v[mm.value + 1] = cmulc(v[mm.value + 1], w);
            w = cmul(w, w1);
          });
        } else {
          uint32_t E = 0;
          static_for<R - 1>([&](auto mm) {
            E += jf;
            if (E >= op.Kf) E -= op.Kf;
            v[mm.value + 1] = cmulc(v[mm.value + 1], twiddle_lds<T>(a, lds, E * op.escale));
          });
        }
      }
      Dft<R, r, true, T>::run(v);
      static_for<R>([&](auto s) { put(s.value, v[s.value]); });
    } else {  // OP_MID: S == 1, j == 0
      Dft<R, r, false, T>::run(v);
      if (m.valid) {
        const int64_t hb = m.gbase - t.off;
        const T hs = (T)a.hscale;
        static_for<R>([&](auto mm) {
          const cx<T> h = ld_g<T>(a.H, hb + (int64_t)digrev<r, g>(mm.value) * a.S_i);
          v[mm.value] = cscale(cmul(v[mm.value], h), hs);
        });
      }
      Dft<R, r, true, T>::run(v);
      static_for<R>([&](auto s) { put(s.value, v[s.value]); });
    }
  }
}

// Register class of a kernel instance: CLS 0 holds the groups with R <= 16,
// CLS 1 every group (R <= 32), both in blocks of up to 256 threads; CLS 2
// the groups with R <= 9 in blocks of up to 1024 threads (at most 128 VGPRs).
// A group's register footprint sets the VGPR count of the whole kernel, so
// the small classes keep occupancy for the common radix-2/4/8 plans, and the
// wide class gives short radix-3/5 groups one item per thread.
template <int R, int CLS>
constexpr bool kind_in_class() { return CLS == 1 || (CLS == 0 && R <= 16) || R <= 9; }

template <int CLS>
constexpr int class_max_threads() { return CLS == 2 ? 1024 : 256; }

template <typename T, int TYPE, int CLS>
__device__ __forceinline__ void dispatch_op(const PassArgs& a, const OpDesc& op,
                                            const TileCtx& t, cx<T>* lds,
                                            const void* in, void* out) {
  switch (op.kind) {
#define PAFC_CASE(id, r, g)                                                          \
  case id:                                                                           \
    if constexpr (kind_in_class<ipow(r, g), CLS>())                                  \
      run_op<T, r, g, TYPE>(a, op, t, lds, in, out);                                 \
    break;
    PAFC_KIND_LIST(PAFC_CASE)
#undef PAFC_CASE
    default:
      break;
  }
}

template <typename T, int CLS>
__device__ __forceinline__ void dispatch_any(const PassArgs& a, const OpDesc& op,
                                             const TileCtx& t, cx<T>* lds,
                                             const void* in, void* out) {
  if (op.type == OP_DIF)
    dispatch_op<T, OP_DIF, CLS>(a, op, t, lds, in, out);
  else if (op.type == OP_DIT)
    dispatch_op<T, OP_DIT, CLS>(a, op, t, lds, in, out);
  else
    dispatch_op<T, OP_MID, CLS>(a, op, t, lds, in, out);
}

// Position of linear tile index x: (i, c).
__device__ __forceinline__ void tile_pos(const PassArgs& a, uint32_t x, uint32_t& i, uint32_t& c) {
  if (a.mode == MODE_STRIDED) {
    i = x >> a.logW;
    c = x & (a.W - 1u);
  } else {
    c = fdiv(x, a.divL);
    i = x - c * a.L;
  }
}

template <typename T>
__device__ __forceinline__ void load_tile(const PassArgs& a, const TileCtx& t,
                                          const void* in, cx<T>* lds) {
  for (uint32_t x = threadIdx.x; x < a.LW; x += blockDim.x) {
    uint32_t i, c;
    tile_pos(a, x, i, c);
    cx<T> v = {(T)0, (T)0};
    if (t.col0 + c < a.ncols) v = ld_g<T>(in, t.base + (int64_t)i * a.S_i + (int64_t)c * a.S_c);
    lds[lds_phys(x, a.lds_sh)] = v;
  }
}

template <typename T>
__device__ __forceinline__ void store_tile(const PassArgs& a, const TileCtx& t,
                                           void* out, const cx<T>* lds) {
  for (uint32_t x = threadIdx.x; x < a.LW; x += blockDim.x) {
    uint32_t i, c;
    tile_pos(a, x, i, c);
    if (t.col0 + c < a.ncols)
      st_g<T>(out, t.base + (int64_t)i * a.S_i + (int64_t)c * a.S_c, lds[lds_phys(x, a.lds_sh)]);
  }
}

// Process tile `tile` of the pass described by `a`; `off` shifts in, out and H
// (the packed offset of a problem in the batched form).
template <typename T, int CLS>
__device__ __forceinline__ void do_tile(const PassArgs& a, const void* in,
                                        void* out, uint32_t tile, int64_t off,
                                        cx<T>* lds) {
  const TileCtx t = make_ctx(a, tile, off);
  if (a.poison) {  // debug: the tile region (below the twiddle copy) is NaN
    const T nan = __builtin_nan("");
    for (uint32_t x = threadIdx.x; x < a.twl_off; x += blockDim.x) lds[x] = cx<T>{nan, nan};
    __syncthreads();
  }
  stage_twiddles<T>(a, lds);
  // load (unless the first op reads global memory itself)
  if (!a.ops[0].src_g) load_tile<T>(a, t, in, lds);
  __syncthreads();  // tile and twiddle tables visible
  const uint32_t nops = a.nops;
  for (uint32_t k = 0; k < nops; ++k) {
    const OpDesc& op = a.ops[k];
    dispatch_any<T, CLS>(a, op, t, lds, in, out);
    if (k + 1 < nops || !op.dst_g) __syncthreads();
  }
  // store (unless the last op wrote global memory itself)
  if (!a.ops[nops - 1].dst_g) store_tile<T>(a, t, out, lds);
}

}  // namespace pafc
