// Persistent, software-pipelined pass kernel for uniform-radix axes.
//
// Same arithmetic as pass_kernel (grouped DIF / DIT stages of the paper's
// transposed and conjugate butterfly kernels, and the fused product with the
// digit-reversed spectrum), specialised at compile time for an axis of
// length L = R^NG split into NG groups of one radix R = r^g.  Each thread owns
// exactly one R-element item of every group.  A block stays resident and
// walks the tiles blockIdx.x, blockIdx.x + gridDim.x, ...; while it
// computes one tile, the global loads of the next tile (its first group's
// inputs and, for the middle pass, its filter values) are already in flight.
// Twiddles are staged once per block in LDS, so no global load other than
// the prefetch sits in the loop and the in-order vector-memory counter never
// makes a group wait on the prefetch.
#pragma once

#include <type_traits>

#include "pass_engine.h"

namespace pafc {

enum { PIPE_FWD = 0, PIPE_INV = 1, PIPE_MID = 2 };

// An axis of NG groups: NG - 1 of radix R and, innermost, one of radix RM
// (RM divides R; RM = R for a uniform axis).  An op of the innermost group
// then runs R / RM groups of RM points per thread, over the thread's R
// consecutive positions, so that every thread still owns one R-point item
// of every op.
template <int R, int NG, int KIND, int RM = R>
struct PipeShape {
  static constexpr int L = ipow(R, NG - 1) * RM;
  static constexpr int NOPS = KIND == PIPE_MID ? 2 * NG - 1 : NG;
  // op i of the pass: its type and its level k (block size K = L / R^k)
  static constexpr int type(int i) {
    return KIND == PIPE_FWD ? OP_DIF
           : KIND == PIPE_INV ? OP_DIT
                              : (i < NG - 1 ? OP_DIF : i == NG - 1 ? OP_MID : OP_DIT);
  }
  static constexpr int level(int i) {
    return KIND == PIPE_FWD ? i : KIND == PIPE_INV ? NG - 1 - i : (i < NG ? i : 2 * NG - 2 - i);
  }
};

struct Item {
  uint32_t c, j, i0;
  bool valid;
};

template <int R, int L, int K, int MODE>
__device__ __forceinline__ Item item_of(uint32_t tid, uint32_t W, uint32_t logW, uint32_t col0,
                                        uint32_t ncols) {
  constexpr uint32_t S = K / R, NB = L / K;
  Item it;
  uint32_t b;
  if (MODE == MODE_STRIDED) {
    it.c = tid & (W - 1u);
    const uint32_t rest = tid >> logW;
    b = rest / S;
    it.j = rest - b * S;
  } else {
    const uint32_t q = tid / S;
    it.j = tid - q * S;
    it.c = q / NB;
    b = q - it.c * NB;
  }
  it.i0 = b * K + it.j;
  it.valid = col0 + it.c < ncols;
  return it;
}

// Two-group forward passes fit two waves per SIMD without spilling and run
// faster when compiled for it; the middle and inverse passes (and longer
// forward ones) need more registers for their prefetch buffers, spill under
// that bound, and keep the compiler's own choice.
template <int KIND, int NG>
constexpr int pipe_waves_per_eu() { return KIND == PIPE_FWD && NG == 2 ? 2 : 1; }

// Threads of one block: one per item, so L W / R of them -- up to 256 for
// the power-of-two shapes, up to 1024 for single radix-3 and radix-5 stages
// (whose items need few registers: a 1024-thread block leaves 128 VGPRs per
// thread); the count need not be a multiple of the wave size.
template <int r, int g>
constexpr int pipe_max_threads() {
  return (r == 3 || r == 5) && g == 1 ? 1024 : r == 3 && g == 2 ? 512 : 256;
}
// FP32 middle passes with folded columns also take 512 threads (a 4096-long
// axis with two columns): their items fit 2 waves per SIMD unspilled; so do
// 4096-long axes in four radix-8 groups (8-point items).
template <typename T, int r, int g, int XC, int NG>
constexpr int pipe_block_limit() {
  return ipow(r, g) == 4 && NG == 6 ? 1024
         : (XC > 0 && sizeof(T) == 4 && !((r == 3 || r == 5) && g == 1)) ||
                 (ipow(r, g) == 8 && NG == 4)
             ? 512
             : pipe_max_threads<r, g>();
}

// Outer pieces of a cut axis (MODE_OUTER) are compiled for the shapes the
// tuned 1-D plans cut off (243 = 3^5 and 625 = 5^4 positions, and the 8-,
// 25- and 27-long pieces of the batched lengths) and the shorter ones of
// cut grid axes (9 = 3^2, 81 = 3^4, 125 = 5^3).
template <int r, int g, int NG>
constexpr bool pipe_outer_shape() {
  return (g == 1 &&
          ((r == 3 && (NG == 2 || NG == 4 || NG == 5)) || (r == 5 && (NG == 3 || NG == 4)))) ||
         (r == 4 && g == 2 && (NG == 1 || NG == 2)) ||  // the 16- and 256-long pieces of long axes
         (r == 3 && g == 2 && NG == 1) ||               // 9-long pieces in one radix-9 group
         (r == 3 && g == 1 && NG == 3) || (r == 5 && g == 1 && NG == 2) ||
         (r == 8 && g == 1 && NG == 1);  // the short outer pieces of the batched 1-D lengths
}

// Long tiles of even length whose items run over consecutive j -- the
// contiguous ones, and the strided ones with folded columns (W = 2^XC <= 4
// columns per row) -- pad their LDS twiddle table (see pipe_kernel); the host
// sizes the table by the same rule.
template <int MODE, int L, int XC>
constexpr bool pipe_tw_pad() {
  return (MODE == MODE_CONTIG || XC > 0) && L % 2 == 0 && L >= 1024;
}

// Butterflies of a 2-point DFT across lane bit b (the two values of a pair
// of lanes differing in bit b): the lower lane keeps x0 + x1, the upper
// x0 - x1.  F_2 is its own conjugate, so the same exchange serves the
// forward and the inverse transform.  The partner's value comes through a
// DPP quad permutation (lanes stay within their group of four).
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL,
                                                            0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, true);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// The DFTs of XC folded axes of length 2 along the columns of a strided tile
// whose row holds exactly those columns (W = 2^XC, column c = lane bits
// 0..XC-1; axis b has column stride 2^b): a butterfly across each of those
// lane bits, for all N values a thread holds.
template <typename T, int XC, int N>
__device__ __forceinline__ void column_dfts(cx<T>* v, uint32_t lane) {
  static_for<XC>([&](auto bc) {
    constexpr int b = decltype(bc)::value;
    constexpr int CTRL = b == 0 ? 0xB1 : 0x4E;  // quad_perm [1,0,3,2] / [2,3,0,1]
    const bool upper = ((lane >> b) & 1u) != 0;
    static_for<N>([&](auto s) {
      const cx<T> p = {dpp_move<CTRL>(v[s.value].re), dpp_move<CTRL>(v[s.value].im)};
      v[s.value] = upper ? csub(p, v[s.value]) : cadd(v[s.value], p);
    });
  });
}

// Digit-reversed slot of value s of a thread's R values in an op at level k
// of an axis of NG groups: the reversal of the op's group, or, for the
// innermost level with groups of RM = r^GM points, of each RM-group.
template <int r, int g, int GM, int NG>
constexpr int slot_rev(int k, int s) {
  return k == NG - 1 ? (s / ipow(r, GM)) * ipow(r, GM) + digrev<r, GM>(s % ipow(r, GM))
                     : digrev<r, g>(s);
}

// PB: the launch runs over many problems of one length through the problem
// table of PassArgs (the batched form's size classes).
template <typename T, int r, int g, int NG, int KIND, int MODE_ARG, int GM = g, int XC = 0,
          bool PB = false>
__global__ void __launch_bounds__((pipe_block_limit<T, r, g, XC, NG>()))
__attribute__((amdgpu_waves_per_eu(pipe_waves_per_eu<KIND, NG>())))
pipe_kernel(const PassArgs* __restrict__ desc, const void* in, void* out) {
  // in and out may be the same array (every pass after the first runs in
  // place), so neither is declared __restrict__
  // an outer piece is a strided pass whose twiddles are those of the whole
  // axis: w_{Kf}^{m jf}, Kf = K jmul, jf = j jmul + (inner position of the
  // column), from the two-level LDS copy of the axis's table
  constexpr bool OUTER = MODE_ARG == MODE_OUTER;
  constexpr int MODE = OUTER ? MODE_STRIDED : MODE_ARG;
  constexpr int R = ipow(r, g);
  // the middle pass's innermost group (RM points; NU of them per thread)
  // and the folded length-2 column axes (strided tiles only)
  constexpr int RM = ipow(r, GM);
  constexpr int NU = R / RM;
  static_assert(GM <= g && R % RM == 0, "innermost group no larger than the others");
  static_assert((GM == g && XC == 0) || (!OUTER && (XC == 0 || MODE == MODE_STRIDED)),
                "short innermost groups: not in outer pieces; folded columns: strided tiles");
  using Sh = PipeShape<R, NG, KIND, RM>;
  constexpr int L = Sh::L;
  constexpr int NOPS = Sh::NOPS;
  constexpr int MID_OP = NG - 1;
  // the first op reads global memory directly unless it is the contiguous
  // inverse (its first group has leg stride 1: load the tile linearly)
  constexpr bool LINEAR_LOAD = (MODE == MODE_CONTIG && KIND == PIPE_INV);
  // the last op writes global memory directly unless it is the contiguous
  // forward (its last group has leg stride 1: store the tile linearly)
  constexpr bool LINEAR_STORE = (MODE == MODE_CONTIG && KIND == PIPE_FWD);

  // Prefetch schedule.  FP64: the next tile's inputs are requested in the
  // first op and the next tile's filter values in the middle op, so both are
  // in flight for a whole tile.  FP32: this tile's filter values in the first
  // op and the next tile's inputs in the last op, which keeps fewer prefetch
  // registers live (measured faster in FP32, slower in FP64).
  constexpr bool PF_LATE = sizeof(T) == 4;
  const PassArgs& a = *desc;
  // LDS slot of tile element x: one pad element every 16 breaks the
  // power-of-two strides.  Tiles of odd length have odd strides and measured
  // fewer bank conflicts unpadded when contiguous (2187- and 3125-long
  // tiles: 4.6 and 5.5 conflict cycles per LDS instruction padded, 2.9
  // unpadded) or strided in FP64 (the 2187^2 middle pass 60.5 -> 58.8 us);
  // strided FP32 tiles (8-byte elements) measured slower unpadded (the 5^9
  // inverse outer pass 20.4 -> 27.3 us) and keep the padding
  auto lphys = [](uint32_t x) -> uint32_t {
    if constexpr (Sh::L % 2 == 1 && (MODE == MODE_CONTIG || sizeof(T) == 16))
      return x;
    else
      return lds_phys(x);
  };
  // LDS slot of twiddle w_L^e.  In a long contiguous tile each op's items
  // run over consecutive j, so an op reads w^(m j (L/K)): strides of m and
  // of 16 m elements, which land on few banks.  One pad element every 16
  // spreads them (the padded table takes L + L / 16 slots).
  auto twp = [](uint32_t e) -> uint32_t {
    if constexpr (pipe_tw_pad<MODE, Sh::L, XC>())
      return e + (e >> 4);
    else
      return e;
  };
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const uint32_t LW = a.LW;
  cx<T>* tw = lds + ((LW + (LW >> 4) + 2) & ~1u);
  const uint32_t tid = threadIdx.x;
  const uint32_t nthr = blockDim.x;
  const uint32_t W = a.W, logW = a.logW;
  const uint32_t ls_i = MODE == MODE_STRIDED ? W : 1u;
  const uint32_t ls_c = MODE == MODE_STRIDED ? 1u : (uint32_t)L;

  if constexpr (OUTER) {
    stage_twiddles<T>(a, lds);  // at a.twl_off == the offset of tw
  } else {
    const cx<T>* lo = reinterpret_cast<const cx<T>*>(a.tw_lo);
    for (uint32_t e = tid; e < (uint32_t)L; e += nthr) tw[twp(e)] = lo[e];
  }
  const uint32_t jmul = a.jmul;
  const bool col_in_j = a.col_in_j != 0;

  // every array this kernel touches is below 4 GiB (the planner checks), so
  // element indices and byte offsets are 32-bit
  const uint32_t S_i = (uint32_t)a.S_i, S_c = (uint32_t)a.S_c, S_o = (uint32_t)a.S_o;
  // Where launch tile t sits: the pass may walk the array backwards, and a
  // batched launch runs over many problems of the same length.  lt is the
  // tile within its problem, base its first element relative to the
  // problem's, pb the problem's first element in the packed arrays, hb that
  // of its filter spectrum in H.
  struct Loc {
    uint32_t lt, col0, base, pb, hb;
  };
  auto locate = [&](uint32_t tile) -> Loc {
    Loc q;
    q.lt = a.rev ? a.ntiles - 1u - tile : tile;
    q.pb = 0;
    q.hb = 0;
    if constexpr (PB) {
      const uint32_t pi = fdiv(q.lt, a.divProb);
      q.lt -= pi * a.tiles_per_prob;
      q.pb = a.prob_off[2 * pi];
      q.hb = a.prob_off[2 * pi + 1];
    }
    const uint32_t o = fdiv(q.lt, a.divTiles);
    q.col0 = (q.lt - o * a.tiles_per_slice) * W;
    q.base = o * S_o + q.col0 * S_c;
    return q;
  };
  auto tile_base = [&](uint32_t tile, uint32_t& col0) -> uint32_t {
    const Loc q = locate(tile);
    col0 = q.col0;
    return q.pb + q.base;
  };

  // prefetch registers: the first op's inputs (or this thread's share of the
  // linear tile load) and, for the middle pass, the filter values of the MID
  // op of the same tile
  cx<T> pre[R];
  cx<T> preh[KIND == PIPE_MID ? R : 1];

  // a.nt selects non-temporal loads for the input (bit 1) and the spectrum
  // (bit 0); the branch is uniform, taken once per tile
  auto fetch_x = [&](uint32_t tile) {
    uint32_t col0;
    const uint32_t base = tile_base(tile, col0);
    auto load = [&](auto nt) {
      constexpr bool NT = decltype(nt)::value;
      if constexpr (LINEAR_LOAD) {
        static_for<R>([&](auto q) {
          const uint32_t x = tid + nthr * q.value;
          const uint32_t c = x / (uint32_t)L, i = x - c * (uint32_t)L;
          pre[q.value] = (col0 + c < a.ncols) ? ld_g32s<T, NT>(in, base + i + c * S_c)
                                              : cx<T>{(T)0, (T)0};
        });
      } else {
        constexpr int k0 = Sh::level(0);
        constexpr int K0 = k0 == NG - 1 ? R : L / ipow(R, k0);
        constexpr int S0 = K0 / R;
        const Item it = item_of<R, L, K0, MODE>(tid, W, logW, col0, a.ncols);
        const uint32_t gb = base + it.i0 * S_i + it.c * S_c;
        static_for<R>([&](auto s) {
          // DIF reads natural positions, DIT reads digit-reversed ones
          constexpr int p = Sh::type(0) == OP_DIT ? slot_rev<r, g, GM, NG>(k0, s.value) : s.value;
          pre[s.value] = it.valid ? ld_g32s<T, NT>(in, gb + (uint32_t)(p * S0) * S_i)
                                  : cx<T>{(T)0, (T)0};
        });
      }
    };
    if (a.nt & 2u) load(std::true_type{}); else load(std::false_type{});
  };
  auto fetch_h = [&](uint32_t tile) {
    if constexpr (KIND == PIPE_MID) {
      // the spectrum has one problem's layout
      const Loc q = locate(tile);
      const Item it = item_of<R, L, R, MODE>(tid, W, logW, q.col0, a.ncols);
      auto load = [&](auto nt) {
        constexpr bool NT = decltype(nt)::value;
        if (a.h_tm) {  // one contiguous block per tile, slot-major
          const uint32_t tb = q.hb + q.lt * LW + tid;
          static_for<R>([&](auto m) {
            preh[m.value] = it.valid ? ld_g32s<T, NT>(a.H, tb + (uint32_t)m.value * nthr)
                                     : cx<T>{(T)0, (T)0};
          });
        } else {
          // slot m = u RM + m2 multiplies frequency m2 of the thread's u-th
          // innermost group, which sits at its digit-reversed position
          const uint32_t gb = q.hb + q.base + it.i0 * S_i + it.c * S_c;
          static_for<R>([&](auto m) {
            constexpr int pos = (m.value / RM) * RM + digrev<r, GM>(m.value % RM);
            preh[m.value] = it.valid ? ld_g32s<T, NT>(a.H, gb + (uint32_t)pos * S_i)
                                     : cx<T>{(T)0, (T)0};
          });
        }
      };
      if (a.nt & 1u) load(std::true_type{}); else load(std::false_type{});
    }
  };

  uint32_t tile = blockIdx.x;
  if (tile < a.ntiles) {
    fetch_x(tile);
    if constexpr (!PF_LATE) fetch_h(tile);
  }
  __syncthreads();  // twiddles visible

  while (tile < a.ntiles) {
    if (a.poison) {  // debug: the tile region (below the twiddles) is NaN
      const T nan = __builtin_nan("");
      for (uint32_t x = tid; x < (uint32_t)(tw - lds); x += nthr) lds[x] = cx<T>{nan, nan};
      __syncthreads();
    }
    const uint32_t next = tile + gridDim.x;
    uint32_t col0;
    const uint32_t base = tile_base(tile, col0);
    if constexpr (LINEAR_LOAD) {
      static_for<R>([&](auto q) { lds[lphys(tid + nthr * q.value)] = pre[q.value]; });
      if constexpr (!PF_LATE)
        if (next < a.ntiles) fetch_x(next);  // pre is free again
      __syncthreads();
    }
    static_for<NOPS>([&](auto opi) {
      constexpr int i = decltype(opi)::value;
      constexpr int type = Sh::type(i);
      constexpr int k = Sh::level(i);
      // an innermost-level op's items are the thread's R consecutive
      // positions (NU groups of RM points)
      constexpr int K = k == NG - 1 ? R : L / ipow(R, k);
      constexpr int S = K / R;
      constexpr bool first = (i == 0) && !LINEAR_LOAD;
      constexpr bool last = (i == NOPS - 1) && !LINEAR_STORE;
      const Item it = item_of<R, L, K, MODE>(tid, W, logW, col0, a.ncols);
      const uint32_t lbase = it.i0 * ls_i + it.c * ls_c;
      const uint32_t gb = base + it.i0 * S_i + it.c * S_c;
      cx<T> v[R];
      // inputs
      static_for<R>([&](auto s) {
        constexpr int p = type == OP_DIT ? slot_rev<r, g, GM, NG>(k, s.value) : s.value;
        if constexpr (first)
          v[s.value] = pre[s.value];
        else
          v[s.value] = lds[lphys(lbase + (uint32_t)(p * S) * ls_i)];
      });
      if constexpr (PF_LATE) {
        // this tile's filter values are loaded while its first ops run; the
        // next tile's inputs while its last op runs.  Each prefetch buffer
        // is live for part of the tile only.
        if constexpr (i == 0) fetch_h(tile);
        if constexpr (i == NOPS - 1)
          if (next < a.ntiles) fetch_x(next);
      } else if constexpr (i == 0 && !LINEAR_LOAD) {
        // the inputs are in registers: start loading the next tile now
        if (next < a.ntiles) fetch_x(next);
      }
      // the twiddles of an outer piece (every op has them: its column's
      // inner position enters the exponent even where S == 1)
      auto outer_tw = [&](auto conj_tag) {
        const uint32_t Kf = (uint32_t)K * jmul;
        const uint32_t esc = a.ops[i].escale;
        const uint32_t jf = it.j * jmul + (col_in_j && it.valid ? fdiv(col0 + it.c, a.divJc) : 0u);
        if (a.twl_global) {
          // the axis's table is too large for LDS: one read of the global
          // (two-level) table, the other twiddles as its powers,
          // w^(m jf) = (w^jf)^m (jf < Kf / R)
          const cx<T> w1 = twiddle<T>(a, jf * esc);
          cx<T> w = w1;
          static_for<R - 1>([&](auto mm) {
            if constexpr (decltype(conj_tag)::value)
              v[mm.value + 1] = cmulc(v[mm.value + 1], w);
            else
              v[mm.value + 1] = cmul(v[mm.value + 1], w);
            w = cmul(w, w1);
          });
          return;
        }
        uint32_t E = 0;
        static_for<R - 1>([&](auto mm) {
          E += jf;
          if (E >= Kf) E -= Kf;
          const cx<T> w = twiddle_lds<T>(a, lds, E * esc);
          if constexpr (decltype(conj_tag)::value)
            v[mm.value + 1] = cmulc(v[mm.value + 1], w);
          else
            v[mm.value + 1] = cmul(v[mm.value + 1], w);
        });
      };
      // folded column axes: their forward DFTs before the first op's own,
      // their inverse DFTs after the last op's (they commute with the
      // stages along the axis)
      if constexpr (XC > 0 && i == 0 && KIND != PIPE_INV) column_dfts<T, XC, R>(v, tid);
      if constexpr (type == OP_DIF) {
        if constexpr (k == NG - 1)
          static_for<NU>([&](auto u) { Dft<RM, r, false, T>::run(v + u.value * RM); });
        else
          Dft<R, r, false, T>::run(v);
        if constexpr (OUTER) {
          outer_tw(std::false_type{});
        } else if constexpr (S > 1) {
          uint32_t E = 0;
          static_for<R - 1>([&](auto mm) {
            E += it.j;
            if (E >= (uint32_t)K) E -= (uint32_t)K;
            v[mm.value + 1] = cmul(v[mm.value + 1], tw[twp(E * (uint32_t)(L / K))]);
          });
        }
      } else if constexpr (type == OP_DIT) {
        if constexpr (OUTER) {
          outer_tw(std::true_type{});
        } else if constexpr (S > 1) {
          uint32_t E = 0;
          static_for<R - 1>([&](auto mm) {
            E += it.j;
            if (E >= (uint32_t)K) E -= (uint32_t)K;
            v[mm.value + 1] = cmulc(v[mm.value + 1], tw[twp(E * (uint32_t)(L / K))]);
          });
        }
        if constexpr (k == NG - 1)
          static_for<NU>([&](auto u) { Dft<RM, r, true, T>::run(v + u.value * RM); });
        else
          Dft<R, r, true, T>::run(v);
      } else {  // MID
        static_for<NU>([&](auto u) { Dft<RM, r, false, T>::run(v + u.value * RM); });
        const T hs = (T)a.hscale;
        static_for<R>([&](auto m) { v[m.value] = cscale(cmul(v[m.value], preh[m.value]), hs); });
        if constexpr (!PF_LATE)
          if (next < a.ntiles) fetch_h(next);
        static_for<NU>([&](auto u) { Dft<RM, r, true, T>::run(v + u.value * RM); });
      }
      if constexpr (XC > 0 && i == NOPS - 1 && KIND != PIPE_FWD) column_dfts<T, XC, R>(v, tid);
      // outputs
      bool tm = false;
      if constexpr (last && KIND == PIPE_FWD && RM == R) tm = a.tm_store != 0;
      if (tm) {
        // the tile-major spectrum order the middle pass reads (PassArgs::h_tm):
        // this last op has the middle op's items (level NG - 1, S = 1), and
        // slot s holds the frequency the middle op's slot s multiplies
        const uint32_t tb = locate(tile).lt * LW + tid;
        static_for<R>([&](auto s) {
          if (it.valid) st_g32<T>(out, tb + (uint32_t)s.value * nthr, v[s.value]);
        });
      } else {
        static_for<R>([&](auto s) {
          // DIF writes frequency m at its digit-reversed position
          constexpr int p = type == OP_DIF ? slot_rev<r, g, GM, NG>(k, s.value) : s.value;
          if constexpr (last) {
            if (it.valid) st_g32<T>(out, gb + (uint32_t)(p * S) * S_i, v[s.value]);
          } else {
            lds[lphys(lbase + (uint32_t)(p * S) * ls_i)] = v[s.value];
          }
        });
      }
      if constexpr (!last) __syncthreads();
    });
    if constexpr (LINEAR_STORE) {
      static_for<R>([&](auto q) {
        const uint32_t x = tid + nthr * q.value;
        const uint32_t c = x / (uint32_t)L, i = x - c * (uint32_t)L;
        if (col0 + c < a.ncols) st_g32<T>(out, base + i + c * S_c, lds[lphys(x)]);
      });
    }
    __syncthreads();  // LDS free for the next tile
    tile = next;
  }
}

// The spectrum in plan layout -> the tile-major order of a middle pass
// (PassArgs::h_tm), for spectra that do not come out of the filter's own
// forward passes (natural-order input, symbols).  Launched with the middle
// pass's descriptor and thread count; slots of columns beyond the edge are
// zero.
template <typename T, int r, int g, int NG, int MODE>
__global__ void __launch_bounds__((pipe_max_threads<r, g>())) pipe_htm_kernel(const PassArgs* __restrict__ desc,
                                                        const void* __restrict__ src,
                                                        void* __restrict__ dst) {
  constexpr int R = ipow(r, g);
  constexpr int L = ipow(R, NG);
  const PassArgs& a = *desc;
  const uint32_t tid = threadIdx.x, nthr = blockDim.x;
  const uint32_t W = a.W, logW = a.logW, LW = a.LW;
  const uint32_t S_i = (uint32_t)a.S_i, S_c = (uint32_t)a.S_c, S_o = (uint32_t)a.S_o;
  for (uint32_t q = blockIdx.x; q < a.ntiles; q += gridDim.x) {
    const uint32_t o = fdiv(q, a.divTiles);
    const uint32_t col0 = (q - o * a.tiles_per_slice) * W;
    const uint32_t base = o * S_o + col0 * S_c;
    const Item it = item_of<R, L, R, MODE>(tid, W, logW, col0, a.ncols);
    const uint32_t gb = base + it.i0 * S_i + it.c * S_c;
    static_for<R>([&](auto m) {
      const cx<T> v = it.valid ? ld_g32<T>(src, gb + (uint32_t)digrev<r, g>(m.value) * S_i)
                               : cx<T>{(T)0, (T)0};
      st_g32<T>(dst, q * LW + (uint32_t)m.value * nthr + tid, v);
    });
  }
}

// ------------------------------------------------------------ instances

#define PAFC_PIPE_SHAPES(X)   \
  X(4, 2, 2) /* L = 256 */    \
  X(4, 2, 3) /* L = 4096 */   \
  X(2, 4, 2) /* L = 256 */    \
  X(2, 4, 3) /* L = 4096 */   \
  X(2, 3, 4) /* L = 4096 in groups of 8 */ \
  X(4, 1, 6) /* L = 4096 in groups of 4 */ \
  X(8, 1, 2) /* L = 64 */     \
  X(8, 1, 3) /* L = 512 */    \
  X(8, 1, 4) /* L = 4096 */   \
  X(4, 2, 1) /* L = 16 */     \
  X(3, 1, 2) /* L = 9 */      \
  X(3, 1, 4) /* L = 81 */     \
  X(3, 1, 5) /* L = 243 */    \
  X(3, 1, 6) /* L = 729 */    \
  X(3, 1, 7) /* L = 2187 */   \
  X(5, 1, 3) /* L = 125 */    \
  X(5, 1, 4) /* L = 625 */    \
  X(5, 1, 5) /* L = 3125 */   \
  X(3, 2, 1) /* L = 9 */      \
  X(3, 2, 3) /* L = 729 */    \
  X(8, 1, 1) /* L = 8 */      \
  X(3, 1, 3) /* L = 27 */     \
  X(5, 1, 2) /* L = 25 */

template <typename T, int r, int g, int NG, bool PB>
const void* pipe_fn(int kind, int mode) {
#define PAFC_PIPE_SEL(K, M) \
  if (kind == K && mode == M) return (const void*)pipe_kernel<T, r, g, NG, K, M, g, 0, PB>;
  PAFC_PIPE_SEL(PIPE_FWD, MODE_CONTIG)
  PAFC_PIPE_SEL(PIPE_FWD, MODE_STRIDED)
  PAFC_PIPE_SEL(PIPE_INV, MODE_CONTIG)
  PAFC_PIPE_SEL(PIPE_INV, MODE_STRIDED)
  PAFC_PIPE_SEL(PIPE_MID, MODE_CONTIG)
  PAFC_PIPE_SEL(PIPE_MID, MODE_STRIDED)
  if constexpr (pipe_outer_shape<r, g, NG>()) {
    PAFC_PIPE_SEL(PIPE_FWD, MODE_OUTER)
    PAFC_PIPE_SEL(PIPE_INV, MODE_OUTER)
  }
#undef PAFC_PIPE_SEL
  return nullptr;
}

// Passes whose innermost group is shorter (GM < g stages) and/or whose
// strided tile row holds XC folded length-2 axes: (r, g, NG, GM, XC), every
// kind (forward, inverse, middle).
#define PAFC_PIPE_EXT_SHAPES(X)                      \
  X(4, 2, 3, 1, 0) /* L = 1024 = 16 x 16 x 4 */      \
  X(4, 2, 3, 1, 1) /* L = 1024, two columns */       \
  X(4, 2, 3, 1, 2) /* L = 1024, four columns */      \
  X(4, 2, 3, 2, 1) /* L = 4096, two columns */       \
  X(4, 2, 2, 2, 1) /* L = 256, two columns */        \
  X(4, 2, 2, 2, 2) /* L = 256, four columns */      \
  X(3, 2, 4, 1, 0) /* L = 2187 = 9 x 9 x 9 x 3 */    \
  X(3, 2, 3, 1, 0) /* L = 243 = 9 x 9 x 3 */

template <typename T, int r, int g, int NG, int GM, int XC, bool PB>
const void* pipe_ext_fn(int kind, int mode) {
#define PAFC_PIPE_EXT_SEL(K)                                                                 \
  if (kind == K) {                                                                           \
    if (mode == MODE_STRIDED) return (const void*)pipe_kernel<T, r, g, NG, K, MODE_STRIDED, GM, XC, PB>; \
    if constexpr (XC == 0)                                                                   \
      if (mode == MODE_CONTIG) return (const void*)pipe_kernel<T, r, g, NG, K, MODE_CONTIG, GM, 0, PB>;  \
  }
  PAFC_PIPE_EXT_SEL(PIPE_FWD)
  PAFC_PIPE_EXT_SEL(PIPE_INV)
  PAFC_PIPE_EXT_SEL(PIPE_MID)
#undef PAFC_PIPE_EXT_SEL
  return nullptr;
}

// The kernel instance for a pass shape (nullptr if none is compiled).  The
// batched instances (PB) exist for the shapes of 1-D plans only: no folded
// column axes.
template <bool PB>
const void* pipe_lookup_t(bool dbl, int r, int g, int ng, int kind, int mode, int gm, int xc) {
  if (gm != g || xc != 0) {
#define PAFC_PIPE_EXT_GO(rr, gg, nn, mm, xx)                                              \
  if constexpr (!PB || xx == 0)                                                           \
    if (r == rr && g == gg && ng == nn && gm == mm && xc == xx)                           \
      return dbl ? pipe_ext_fn<double, rr, gg, nn, mm, xx, PB>(kind, mode)                \
                 : pipe_ext_fn<float, rr, gg, nn, mm, xx, PB>(kind, mode);
    PAFC_PIPE_EXT_SHAPES(PAFC_PIPE_EXT_GO)
#undef PAFC_PIPE_EXT_GO
    return nullptr;
  }
#define PAFC_PIPE_GO(rr, gg, nn)                                                          \
  if (r == rr && g == gg && ng == nn)                                                     \
    return dbl ? pipe_fn<double, rr, gg, nn, PB>(kind, mode)                              \
               : pipe_fn<float, rr, gg, nn, PB>(kind, mode);
  PAFC_PIPE_SHAPES(PAFC_PIPE_GO)
#undef PAFC_PIPE_GO
  return nullptr;
}

}  // namespace pafc
