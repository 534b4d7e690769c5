// Internal descriptors shared by the host planner and the gfx950 kernels.
//
// A "pass" is one kernel launch that reads every element of the array once
// from HBM, applies a sequence of "ops" to tiles held in LDS, and writes every
// element once.  A tile is L x W elements: L consecutive positions along the
// (virtual) axis being transformed, times W columns.  Each op is one group of
// g consecutive radix-r stages of the paper's stage sequence (R = r^g):
//
//   DIF op (forward, A^T; Alg. alg:transposed-butterfly-kernel grouped):
//     for every block b and offset j < S = K/R, the R elements at
//     b*K + j + s*S (s < R) are replaced by an R-point DFT over s; frequency m
//     is written to position b*K + j + digrev(m)*S after multiplication by the
//     twiddle w_K^{m j}.  digrev is the base-r reversal of g digits.  This is
//     exactly g stages of B_{r,k}^T (eq. 25 transposed), stage k = K first.
//   DIT op (inverse, conj A; Alg. alg:butterfly-related-kernel grouped): the
//     mirror image: read position digrev(m), multiply by conj(w_K^{m j}),
//     inverse R-point DFT, write natural position s.
//   MID op: the innermost DIF group (S = 1, no twiddle), the product with the
//     filter spectrum at the same digit-reversed positions, and the innermost
//     DIT group, without leaving registers (the point of eq. 35: both
//     operands of the product share one digit-reversed order).
#pragma once

#include <stdint.h>

namespace pafc {

enum { MODE_CONTIG = 0, MODE_STRIDED = 1 };
// Pipelined kernel only: a strided outer piece of a cut axis, whose twiddles
// are those of the whole axis (two-level LDS table, exponent with the
// column's inner position); its PassArgs::mode stays MODE_STRIDED.
enum { MODE_OUTER = 2 };
enum { OP_DIF = 0, OP_DIT = 1, OP_MID = 2 };

// Group kinds (r, g) instantiated in the kernels.
#define PAFC_KIND_LIST(X) \
  X(0, 2, 1)              \
  X(1, 2, 2)              \
  X(2, 2, 3)              \
  X(3, 2, 4)              \
  X(4, 2, 5)              \
  X(5, 4, 1)              \
  X(6, 4, 2)              \
  X(7, 8, 1)              \
  X(8, 3, 1)              \
  X(9, 3, 2)              \
  X(10, 3, 3)             \
  X(11, 5, 1)             \
  X(12, 5, 2)

constexpr int kNumKinds = 13;
constexpr int kMaxOps = 12;
// most blocks of the Rader route's sum kernel (its partial-sum buffer)
constexpr unsigned kRaderBlocks = 1024;

// Unsigned 32-bit division by an invariant divisor d >= 1 (Granlund and
// Montgomery's multiply-high method): q = (umulhi(x, m) + x) >> l with
// l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1; exact for all x < 2^32.
struct FastDiv {
  uint32_t d;
  uint32_t m;
  uint32_t l;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  f.l = l;
  f.m = (uint32_t)((((1ull << l) - d) << 32) / d + 1);
  return f;
}

struct OpDesc {
  int32_t type;     // OP_DIF / OP_DIT / OP_MID
  int32_t kind;     // index in PAFC_KIND_LIST
  int32_t R;        // group radix r^g
  int32_t tw;       // 1 if external twiddles are needed
  uint32_t K;       // local block size (positions along the virtual axis)
  uint32_t S;       // leg stride K / R
  uint32_t nitems;  // items per tile = (L / R) * W
  uint32_t Kf;      // block size of the full transform = K * jmul
  uint32_t escale;  // twiddle-table exponent scale = n_tw / Kf
  uint16_t src_g;   // 1: the op reads its inputs straight from global memory
  uint16_t dst_g;   // 1: the op writes its outputs straight to global memory
  FastDiv divS;     // division by S
  FastDiv divNB;    // division by L / K (blocks per column)
  // Column op: the whole DFT of a short axis folded into a strided pass,
  // whose tile row holds every column (W == ncols, row-major columns of the
  // faster axes).  Its legs are columns p*cs + lo within a block of R*cs
  // columns; no twiddles, LDS in and out.
  uint32_t cross;   // 1 for a column op
  uint32_t cs;      // column stride of the folded axis within a row
  FastDiv divQ;     // division by W / R (column groups per row)
  FastDiv divCs;    // division by cs
};

struct PassArgs {
  const void* H;       // filter spectrum for OP_MID (same layout as the data)
  double hscale;       // OP_MID multiplies by H * hscale (1/N: the spectrum is
                       // kept unscaled)
  const void* tw_lo;   // twiddle table(s): w_{n_tw}^E
  const void* tw_hi;   // second level (NULL for a flat table)
  uint32_t tw_bits;    // E = lo + (hi << tw_bits) when two-level
  uint32_t mode;       // MODE_CONTIG / MODE_STRIDED
  uint32_t L;          // positions along the virtual axis
  uint32_t W;          // columns per tile (power of two)
  uint32_t logW;
  uint32_t LW;         // L * W
  int64_t S_i;         // element stride between consecutive positions
  int64_t S_c;         // element stride between consecutive columns
  int64_t S_o;         // element stride between outer slices
  uint32_t ncols;      // columns per slice (the last tile may be partial)
  uint32_t tiles_per_slice;
  uint32_t ntiles;
  uint32_t jmul;       // j of the full transform = j * jmul + column / divJc.d
  uint32_t col_in_j;   // 1 when the column index enters the twiddle exponent
  uint32_t nops;
  FastDiv divL;        // division by L
  FastDiv divTiles;    // division by tiles_per_slice
  FastDiv divJc;       // column -> inner position of an outer piece (the
                       // stride of the axis; 1 for a 1-D transform)
  uint32_t twl_bits;   // LDS copy of the twiddles: w^E = lo[E & (2^b - 1)] * hi[E >> b]
  uint32_t twl_nhi;    // entries of the hi table (the lo table has 2^twl_bits)
  uint32_t twl_off;    // element offset of the LDS tables after the tile
  uint32_t twl_global; // 1: no LDS copy (it would not fit beside the tile);
                       // twiddles are read from the global table
  uint32_t rev;        // 1: tile t of the launch is tile ntiles - 1 - t (the
                       // pass walks the array from its end)
  uint32_t h_tm;       // middle pass: H is stored tile-major -- the value
                       // thread t takes for frequency slot m of (logical) tile
                       // q sits at q * LW + m * threads + t, so each tile's
                       // spectrum is one contiguous block read in order
  uint32_t tm_store;   // forward pass: its last op writes that tile-major
                       // order (the filter's last forward pass)
  uint32_t lds_sh;     // LDS padding of the general engine: one pad element
                       // every 2^lds_sh (4: breaks power-of-two strides), or
                       // none (31) for contiguous tiles of odd length, whose
                       // strides are odd and conflict-free unpadded
  uint32_t poison;     // debug: fill the LDS tile with NaN before each tile,
                       // so a read of LDS that no op wrote shows in the result
  uint32_t nt;         // pipelined kernel: bit 0 reads the spectrum, bit 1
                       // the pass's input, with non-temporal loads (set for
                       // arrays too large to stay in the last-level cache,
                       // where such a read would only evict lines that the
                       // next pass could still use)
  // one launch over many problems of one length (the batched form's size
  // classes, pipelined kernel only): launch tile t is tile t mod
  // tiles_per_prob of problem t / tiles_per_prob, whose data start at element
  // prob_off[2 q] of the packed arrays and whose filter spectrum at element
  // prob_off[2 q + 1] of H.  NULL for a single problem.
  const uint32_t* prob_off;
  uint32_t tiles_per_prob;
  FastDiv divProb;
  OpDesc ops[kMaxOps];
};

// Tiles of the batched launch: a pass over one tile of one problem.
struct BatchTile {
  uint32_t desc;    // index of the PassArgs template (size class + pass)
  uint32_t tile;    // tile index within that problem's pass
  int64_t offset;   // element offset of the problem in the packed arrays
};

// Jobs of the persistent batched launch: one whole problem, all of its
// passes, run by the block that claims it.
struct BatchJob {
  uint32_t desc;    // index of the PassArgs of its first pass; the others follow
  uint32_t npass;   // passes of its size class
  int64_t offset;   // element offset of the problem in the packed arrays
};

// Control words of the persistent batched launch (zero between launches).
struct BatchCtl {
  uint32_t next;    // next job to claim
  uint32_t exited;  // blocks that have left the claim loop
};

}  // namespace pafc
