// Host side of libpafc: planner, twiddle generation, and the C ABI of
// include/pafc.h.
//
// The plan follows the paper's formulation of the convolution without index
// reversal (eq. 35; d-way form in Sec. "Permutation-avoiding
// multi-dimensional convolution"; mixed radix in Sec. "Mixed-radix
// framework"): per axis a radix sequence rho = [r_1, ..., r_t] (r_1 the
// innermost stage), the forward transform A^T applied stage r_t first, the
// inverse conj(A) stage r_1 first.  The planner only decides how those stages
// are cut into HBM passes and register groups; it never changes the stages.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pafc.h"
#include "pafc_internal.h"

// Device memory of pafc_convolve_with_filter_noalloc: the per-call filter
// spectrum.  Every device the library runs on holds its own copy from module
// load to process exit.  In host code the name is only a host-side stand-in:
// host code uses the address hipGetSymbolAddress returns for the current
// device (scratch_address below), never the name.
static __device__ __align__(256) unsigned char scratch[PAFC_NOALLOC_MAX_BYTES];

namespace pafc {
hipError_t launch_pass(bool dbl, int cls, const PassArgs* d_desc, uint32_t ntiles, const void* in,
                       void* out, uint32_t threads, size_t lds_bytes, hipStream_t s);
int batch_persist_blocks_per_cu(bool dbl, size_t lds_bytes);
hipError_t launch_batch_persist(bool dbl, const PassArgs* descs, const BatchJob* jobs,
                                uint32_t njobs, BatchCtl* ctl, uint32_t grid, size_t lds_bytes,
                                const void* in, void* out, hipStream_t s);
hipError_t launch_batch(bool dbl, int cls, const PassArgs* descs, const BatchTile* tiles,
                        uint32_t first, uint32_t count, const void* in, void* out,
                        uint32_t threads, size_t lds_bytes, hipStream_t s);
hipError_t launch_scale(bool dbl, void* p, int64_t n, double s, hipStream_t st);
bool pipe_supported(int r, int g, int ng);
bool pipe_outer_supported(int r, int g, int ng);
bool pipe_ext_supported(int r, int g, int ng, int gm, int xc, int kind, int mode);
int pipe_thread_limit(int r, int g, bool dbl = true, int xc = 0);
int pipe_uniform_threads(int r, int g, int ng);

int pipe_blocks_per_cu(bool dbl, int r, int g, int ng, int kind, int mode, uint32_t threads,
                       size_t lds, int gm, int xc);
hipError_t launch_pipe_htm(bool dbl, int r, int g, int ng, int mode, const PassArgs* d,
                           uint32_t ntiles, uint32_t threads, const void* src, void* dst,
                           hipStream_t s);
hipError_t launch_pipe(bool dbl, int r, int g, int ng, int kind, int mode, const PassArgs* d,
                       uint32_t grid, uint32_t threads, size_t lds, const void* in, void* out,
                       hipStream_t s, int gm, int xc, hipEvent_t t0 = nullptr,
                       hipEvent_t t1 = nullptr);
int pipe_batch_blocks_per_cu(bool dbl, int r, int g, int ng, int kind, int mode,
                             uint32_t threads, size_t lds, int gm);
hipError_t launch_pipe_batch(bool dbl, int r, int g, int ng, int kind, int mode, int gm,
                             const PassArgs* d, uint32_t grid, uint32_t threads, size_t lds,
                             const void* in, void* out, hipStream_t s);
hipError_t launch_mul(bool dbl, const void* x, const void* h, void* y, int64_t n, double s,
                      bool nt_h, hipStream_t st);
hipError_t launch_stream_copy(int kind, const void* src, void* dst, int64_t n16, hipStream_t st);
hipError_t launch_pfa_gather(bool dbl, const void* in, void* out, const uint32_t* t0,
                             const uint32_t* t1, const uint32_t* t2, uint32_t N1, uint32_t N2,
                             uint32_t n, hipStream_t st);
hipError_t launch_pfa_map(bool dbl, int dir, const void* in, void* out, uint32_t N0, uint32_t N1,
                          uint32_t N2, uint32_t uinv, hipStream_t st);
hipError_t launch_bluestein(bool dbl, int stage, const void* src, const void* c, void* dst,
                            const void* hn, int64_t n, int64_t m, double s, hipStream_t st);
hipError_t launch_rader(bool dbl, int stage, int mode, const void* src, const void* x, void* dst,
                        void* hq, const uint32_t* pw, const uint32_t* lg, double* part,
                        void* consts, uint32_t p, double s, hipStream_t st);
hipError_t launch_symbol(bool dbl, void* H, const void* g, const int32_t* m0, const int32_t* m1,
                         const int32_t* m2, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t off0,
                         uint32_t off1, uint32_t off2, int mode, hipStream_t st);
hipError_t launch_permute_rows(bool dbl, const void* in, void* out, const void* h,
                               const int32_t* m0, const int32_t* m1, const int32_t* mlast,
                               uint32_t n0, uint32_t n1, uint32_t nlast, uint32_t rows_per_block,
                               double s, bool nt_h, hipStream_t st);
hipError_t launch_permute_gather(bool dbl, const void* in, void* out, const void* h,
                                 const int32_t* m0, const int32_t* m1, const int32_t* m2,
                                 uint32_t n0, uint32_t n1, uint32_t n2, double s, bool nt_h,
                                 hipStream_t st);
hipError_t launch_permute_tile(bool dbl, const void* in, void* out, const void* h,
                               const int32_t* m0, const int32_t* m1, const int32_t* mlast,
                               uint32_t n0, uint32_t n1, uint32_t log_nl, double s, bool nt_h,
                               hipStream_t st);
}  // namespace pafc

using namespace pafc;

namespace {

constexpr size_t kLdsBudget = 160 * 1024;  // LDS per CU on gfx950
// Planner knobs read at plan time (autotuning and experiments):
//   PAFC_TUNE_IO  bit mask of direct global I/O: 1 contiguous-tile loads,
//                 2 contiguous-tile stores, 4 strided-tile loads, 8 strided-
//                 tile stores (default 13: all but contiguous stores)
//   PAFC_TUNE_WC / PAFC_TUNE_WS  tile width of contiguous / strided tiles
//   PAFC_TUNE_MID  axis that carries the fused product (default 0, the slowest)
//   PAFC_WIDE      0 disables the wide (1024-thread) register class
//   PAFC_FOLD      0 keeps short faster axes in passes of their own
//   PAFC_SNAKE     0 walks every pass's tiles in the same direction
//   PAFC_AXIS_ORDER 1 runs the other axes' forward passes slowest first
//   PAFC_HTM       0 keeps the spectrum in plan layout (no tile-major order)
//   PAFC_LLC_MB    array size in MiB from which the spectrum and a sequence's
//                  input are read non-temporally (default 256; 1 << 20 never)
//   PAFC_PIPE      0 runs every pass on the general engine (no pipelined kernel)
//   PAFC_PIPE_OUTER 0 keeps outer pieces of cut axes on the general engine
//   PAFC_TUNE_GMAX3 / PAFC_TUNE_GMAX5  largest radix-3 / radix-5 register
//                  group (stages) where the tuning table has no entry
//   PAFC_NO_TUNING_TABLE 1 (binding) loads no tuning table
//   PAFC_LDS_POISON 1 (debug) every pass fills its LDS tile with NaN first
//   PAFC_BATCH_STREAMS streams of the batched classes form (default 6)
//   PAFC_BATCH_LDS_KB  tile LDS bound of the batched persistent form
//   PAFC_LDS_PAD   1 pads the LDS tiles of odd-length contiguous passes too
//   PAFC_FAULT_INJECT=oom  pafc_plan fails with OUT_OF_MEMORY after its first
//                  allocations (tests of the cleanup path)
//   PAFC_BLUESTEIN 1 plans a prime length by Bluestein's method even where
//                  Rader's applies (p - 1 {2,3,5}-smooth)
int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  return v && *v ? atoi(v) : dflt;
}
constexpr uint32_t kMaxThreads = 256;       // register classes 0 and 1
constexpr uint32_t kMaxWideThreads = 1024;  // register class 2 (groups R <= 9)

// ------------------------------------------------------------- tuning table

struct TuneKey {
  int dtype;
  int64_t n;
  bool operator<(const TuneKey& o) const { return dtype != o.dtype ? dtype < o.dtype : n < o.n; }
};
struct TuneVal {
  int64_t split = 0;  // inner length of a two-level 1-D transform (0 = default)
  int W = 0;          // tile width of the axis (inner piece when split; 0 = default)
  int Wo = 0;         // tile width of the outer piece of a split 1-D transform
  int gmax3 = 0;      // largest group of radix-3 stages (0 = default)
  int gmax5 = 0;      // largest group of radix-5 stages (0 = default)
  int gmax3i = 0;     // the same for the inner pieces of a cut axis (0 = gmax3)
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

bool tune_lookup(int dtype, int64_t n, TuneVal* v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find({dtype, n});
  if (it == g_tune.end()) return false;
  *v = it->second;
  return true;
}

// ------------------------------------------------------------- radix / pos

int64_t ipow64(int64_t b, int e) {
  int64_t r = 1;
  while (e-- > 0) r *= b;
  return r;
}

// Group kinds available to the kernels: (r, g) -> kind id.
int kind_of(int r, int g) {
  static const int tbl[][3] = {
#define PAFC_ROW(id, rr, gg) {id, rr, gg},
      PAFC_KIND_LIST(PAFC_ROW)
#undef PAFC_ROW
  };
  for (auto& t : tbl)
    if (t[1] == r && t[2] == g) return t[0];
  return -1;
}

int env_int(const char* name, int dflt);

// Largest group of consecutive radix-r stages fused into one register op.
// Groups with R > 16 need the large register class of the kernels.
struct GroupCaps {
  int g2 = 4;  // R = 16 (8 with 3)
  int g4 = 2;  // R = 16 (4 with 1)
  int g3 = 3;  // R = 27 (9 with 2)
  int g5 = 2;  // R = 25 (5 with 1)
  int lim3 = 0;  // a caller's bound on g3 (0: none)
};

int gmax_of(int r, const GroupCaps& gc) {
  switch (r) {
    case 2: return gc.g2;
    case 4: return gc.g4;
    case 8: return 1;  // R = 8
    case 3: return gc.g3;
    case 5: return gc.g5;
  }
  return 1;
}

// Planner's radix sequence for n (innermost first): radix-4 stages for the
// power of two (one radix-8 stage absorbs an odd exponent >= 3, a lone 2
// otherwise), then radix 3, then radix 5.
bool auto_rho(int64_t n, std::vector<int>* rho) {
  rho->clear();
  int a = 0, b = 0, c = 0;
  while (n % 2 == 0) { n /= 2; ++a; }
  while (n % 3 == 0) { n /= 3; ++b; }
  while (n % 5 == 0) { n /= 5; ++c; }
  if (n != 1) return false;
  if (a % 2 == 1) {
    if (a >= 3) { rho->push_back(8); a -= 3; }
    else { rho->push_back(2); a -= 1; }
  }
  for (int i = 0; i < a / 2; ++i) rho->push_back(4);
  for (int i = 0; i < b; ++i) rho->push_back(3);
  for (int i = 0; i < c; ++i) rho->push_back(5);
  // keep equal radices adjacent: innermost the radix-4 run, then the lone
  // 2/8, so that the radix-4 stages group into R = 16 ops
  std::stable_sort(rho->begin(), rho->end(), [](int x, int y) {
    auto key = [](int r) { return r == 4 ? 0 : r == 8 ? 1 : r == 2 ? 2 : r == 3 ? 3 : 4; };
    return key(x) < key(y);
  });
  return true;
}

// Mixed-radix digit reversal: with k = d_t + r_t (d_{t-1} + ... + r_2 d_1),
// pos(k) = d_1 + r_1 (d_2 + ... + r_{t-1} d_t); entry pos(k) of A^T x holds
// entry k of F x (consequence of F = P_rho A_rho^T, Sec. "Mixed-radix
// framework").
std::vector<int32_t> pos_table(int64_t n, const std::vector<int>& rho) {
  const int t = (int)rho.size();
  std::vector<int32_t> out((size_t)n);
  std::vector<int> d(t);
  for (int64_t k = 0; k < n; ++k) {
    int64_t x = k;
    for (int i = t - 1; i >= 0; --i) { d[i] = (int)(x % rho[i]); x /= rho[i]; }
    int64_t p = 0;
    for (int i = t - 1; i >= 0; --i) p = p * rho[i] + d[i];
    out[(size_t)k] = (int32_t)p;
  }
  return out;
}

// ---------------------------------------------------------------- twiddles

// w_n^E = exp(-2 pi i E / n) in FP64, from long double.  The angle
// theta = 2 pi E / n is reduced exactly in integers to an octant o and a
// remainder r (8E = o n + r); cosl/sinl are only evaluated on [0, pi/4]
// (phi = (pi/4) r / n, or its reflection (pi/4)(n - r)/n in the odd
// octants), and the octant is applied by exact swaps and sign changes.  So
// +-1 and +-i are exact, (+-1 +-i)/sqrt(2) correctly rounded, and
// w_n^(n-E) is exactly the conjugate of w_n^E.
void omega64(int64_t n, int64_t E, double* re, double* im) {
  E %= n;
  if (E < 0) E += n;
  const __int128 num = (__int128)8 * E;
  const int o = (int)(num / n);
  const int64_t r = (int64_t)(num - (__int128)o * n);
  const long double pi4 = 0.785398163397448309615660845819875721L;
  const int64_t rr = (o & 1) ? n - r : r;  // odd octants: reflected remainder
  long double c, sn;
  if (rr == 0) {
    c = 1.0L;
    sn = 0.0L;
  } else if (rr == n) {
    c = sn = 0.707106781186547524400844362104849039L;
  } else {
    const long double phi = (long double)rr / (long double)n * pi4;
    c = cosl(phi);
    sn = sinl(phi);
  }
  // (cos theta, sin theta) from (c, sn) = (cos, sin) of phi or its reflection
  long double ct, st;
  switch (o) {
    case 0: ct = c; st = sn; break;
    case 1: ct = sn; st = c; break;
    case 2: ct = -sn; st = c; break;
    case 3: ct = -c; st = sn; break;
    case 4: ct = -c; st = -sn; break;
    case 5: ct = -sn; st = -c; break;
    case 6: ct = sn; st = -c; break;
    default: ct = c; st = -sn; break;
  }
  *re = (double)ct;
  *im = (double)(-st);
}

struct TwTable {
  int64_t n = 0;
  int64_t lo_off = 0, hi_off = -1;  // element offsets in the plan's table buffer
  uint32_t bits = 0;
};

// ---------------------------------------------------------------- planning

struct Seg {  // one pass-sized piece of an axis transform
  uint32_t mode = MODE_CONTIG, L = 0, W = 1;
  int64_t S_i = 1, S_c = 1, S_o = 0;
  uint32_t ncols = 1, nouter = 1, jmul = 1, col_in_j = 0;
  uint32_t jcdiv = 1;  // column -> inner position of an outer piece
  int64_t n_tw = 0;
  bool tw_global = false;  // twiddles from the global table, no LDS copy
  std::vector<int> rho;  // this piece's stages, innermost first
  GroupCaps caps;
  size_t lds = kLdsBudget;  // LDS one tile of the piece may use
};

struct Pass {
  int kind = 0;  // 0 = pass kernel, 1 = mul, 2 = permute, 3 = scale
  PassArgs a;
  uint32_t threads = 0;
  size_t lds = 0;
  int cls = 0;
  int64_t tw_n = 0;
  bool mid = false;
  // permute / mul details
  int perm_dir = 0;  // 1: dr -> nat (with product), 2: nat -> dr
  uint32_t desc = 0;  // index of the uploaded descriptor
  // pipelined persistent kernel (uniform-radix axis, one item per thread)
  bool pipe = false;
  int pipe_r = 0, pipe_g = 0, pipe_ng = 0, pipe_kind = 0;
  int pipe_mode = 0;  // MODE_CONTIG, MODE_STRIDED, or MODE_OUTER (an outer piece)
  int pipe_gm = 0;    // stages of the innermost group (a middle pass's may be fewer)
  int pipe_xc = 0;    // folded length-2 column axes of a strided middle pass
  uint32_t pipe_grid = 0;
  uint32_t pipe_threads = 0;  // one per item (the general engine's count is `threads`)
  size_t pipe_lds = 0;

  std::string label;
};

struct AxisInfo {
  int64_t n = 0;
  std::vector<int> rho;
  std::vector<Seg> segs;
  std::vector<int32_t> pos, posinv;
};

struct PlanCore {
  int ndim = 0;
  int64_t dims[3] = {1, 1, 1};
  int dtype = PAFC_C128;
  int variant = PAFC_PERM_FREE;
  int64_t N = 0;
  size_t elem = 16;
  int middle = 0;
  std::vector<AxisInfo> axes;
  std::vector<Pass> conv, fwd, inv;
  std::map<int64_t, TwTable> tw;
  int64_t tw_elems = 0;
  int64_t hbm_conv = 0, hbm_fwd = 0;
};

std::vector<std::pair<int, int>> group_runs(const std::vector<int>& rho_inner_first,
                                            const GroupCaps& gc) {
  // DIF order: outermost stage (last entry) first; equal radices grouped.
  std::vector<std::pair<int, int>> out;
  std::vector<int> st(rho_inner_first.rbegin(), rho_inner_first.rend());
  size_t i = 0;
  while (i < st.size()) {
    size_t j = i;
    while (j < st.size() && st[j] == st[i]) ++j;
    const int r = st[i];
    const int t = (int)(j - i);
    const int gm = gmax_of(r, gc);
    const int G = (t + gm - 1) / gm;
    for (int q = 0; q < G; ++q) {
      int g = t / G + (q < t % G ? 1 : 0);
      out.push_back({r, g});
    }
    i = j;
  }
  return out;
}

uint32_t ilog2u(uint32_t w) {
  uint32_t l = 0;
  while ((1u << l) < w) ++l;
  return l;
}

size_t tile_lds_bytes(uint64_t LW, size_t elem) { return (size_t)(LW + (LW >> 4) + 1) * elem; }

uint32_t pow2_floor(uint64_t x) {
  uint32_t p = 1;
  while ((uint64_t)p * 2 <= x) p *= 2;
  return p;
}

// Bytes of the LDS two-level twiddle copy of a piece (see make_pass).
size_t twl_bytes(int64_t n_tw, size_t elem) {
  uint32_t b = 0;
  while (((int64_t)1 << (2 * b)) < n_tw) ++b;
  const int64_t nhi = (n_tw + ((int64_t)1 << b) - 1) >> b;
  return (size_t)(((int64_t)1 << b) + nhi + 2) * elem;
}

void choose_width(Seg& s, size_t elem, int tuneW) {
  // ~4096 elements per tile; strided tiles also want >= 256 B row segments
  uint32_t W = pow2_floor(std::max<uint64_t>(1, 4096 / std::max<uint32_t>(1, s.L)));
  if (s.mode == MODE_STRIDED) W = std::max<uint32_t>(W, 16);
  // contiguous tiles of very short axes take more pencils (whole 4096-element
  // tiles); other tiles stay within 256 columns
  W = std::min<uint32_t>(W, s.mode == MODE_CONTIG && s.L < 16 ? 4096u : 256u);
  W = std::min<uint32_t>(W, pow2_floor(std::max<uint64_t>(1, s.ncols)));
  if (tuneW > 0) W = pow2_floor((uint64_t)tuneW);
  const int envW = env_int(s.mode == MODE_STRIDED ? "PAFC_TUNE_WS" : "PAFC_TUNE_WC", 0);
  if (envW > 0) W = std::min<uint32_t>(pow2_floor((uint64_t)envW),
                                       pow2_floor(std::max<uint64_t>(1, s.ncols)));
  const size_t tw = s.tw_global ? 0 : twl_bytes(s.n_tw, elem);
  while (W > 1 && tile_lds_bytes((uint64_t)s.L * W, elem) + tw > s.lds) W /= 2;
  s.W = W;
}

bool fits_lds(int64_t L, size_t elem, size_t budget) {
  return tile_lds_bytes((uint64_t)L, elem) <= budget;
}

// A piece reads its twiddles from the global (L2-resident) table instead of
// an LDS copy when the copy would not fit beside a one-column tile, or when
// it is larger than 64 KB (PAFC_TUNE_TWG bytes): staging it would cost more
// than the tile's own data (measured: 2^24-long axes twice as fast with
// global reads, the 48 KB tables of 5^9 faster in LDS).
bool twiddles_global(int64_t L, int64_t n_tw, size_t elem, size_t budget) {
  const size_t tw = twl_bytes(n_tw, elem);
  const int lim = env_int("PAFC_TUNE_TWG", 64 * 1024);
  return tile_lds_bytes((uint64_t)L, elem) + tw > budget || (lim > 0 && tw > (size_t)lim);
}

// Build the op list of one pass over segment s.  kind: 0 = DIF only,
// 1 = DIT only, 2 = DIF..., MID, ...DIT.
// A short axis folded into a strided pass as a column op (see OpDesc).
struct CrossAxis {
  int r, g;     // its one register group: R = r^g = its length
  uint32_t cs;  // its column stride within a tile row
};

bool build_ops(const Seg& s, int kind, PassArgs& a, int* cls,
               const std::vector<CrossAxis>* cross = nullptr) {
  auto groups = group_runs(s.rho, s.caps);
  struct G { int r, g, R; uint32_t K, S; };
  std::vector<G> gs;
  uint32_t K = s.L;
  for (auto& pr : groups) {
    int R = (int)ipow64(pr.first, pr.second);
    G g{pr.first, pr.second, R, K, K / (uint32_t)R};
    gs.push_back(g);
    K /= (uint32_t)R;
  }
  if (K != 1) return false;
  *cls = 0;
  auto mk = [&](const G& g, int type) {
    OpDesc op;
    memset(&op, 0, sizeof(op));
    op.type = type;
    op.kind = kind_of(g.r, g.g);
    op.R = g.R;
    op.K = g.K;
    op.S = g.S;
    op.tw = (g.S > 1 || s.col_in_j) ? 1 : 0;
    op.nitems = (s.L / (uint32_t)g.R) * s.W;
    op.Kf = g.K * s.jmul;
    op.escale = (uint32_t)(s.n_tw / ((int64_t)g.K * s.jmul));
    op.divS = make_fastdiv(g.S);
    op.divNB = make_fastdiv(s.L / g.K);
    if (g.R > 16) *cls = 1;
    return op;
  };
  auto mkx = [&](const CrossAxis& x, int type) {
    OpDesc op;
    memset(&op, 0, sizeof(op));
    op.type = type;
    op.kind = kind_of(x.r, x.g);
    op.R = (int32_t)ipow64(x.r, x.g);
    op.K = (uint32_t)op.R;
    op.S = 1;
    op.tw = 0;
    op.nitems = s.L * (s.W / (uint32_t)op.R);
    op.divS = make_fastdiv(1);
    op.divNB = make_fastdiv(1);
    op.cross = 1;
    op.cs = x.cs;
    op.divQ = make_fastdiv(s.W / (uint32_t)op.R);
    op.divCs = make_fastdiv(x.cs);
    if (op.R > 16) *cls = 1;
    return op;
  };
  std::vector<OpDesc> ops;
  const bool folded = cross && !cross->empty();
  // folded short axes: their forward DFTs before the pass's own forward
  // stages, their inverse DFTs after its inverse stages
  if (folded) {
    if (s.mode != MODE_STRIDED || s.W != s.ncols) return false;
    if (kind != 1)
      for (auto& x : *cross) ops.push_back(mkx(x, OP_DIF));
  }
  if (kind == 0) {
    for (auto& g : gs) ops.push_back(mk(g, OP_DIF));
  } else if (kind == 1) {
    for (auto it = gs.rbegin(); it != gs.rend(); ++it) ops.push_back(mk(*it, OP_DIT));
  } else {
    for (size_t i = 0; i + 1 < gs.size(); ++i) ops.push_back(mk(gs[i], OP_DIF));
    ops.push_back(mk(gs.back(), OP_MID));
    for (size_t i = gs.size() - 1; i-- > 0;) ops.push_back(mk(gs[i], OP_DIT));
  }
  if (folded && kind != 0)
    for (auto it = cross->rbegin(); it != cross->rend(); ++it) ops.push_back(mkx(*it, OP_DIT));
  if ((int)ops.size() > kMaxOps) return false;
  for (auto& op : ops)
    if (op.kind < 0) return false;
  // Direct global I/O for the first and last op where it stays coalesced:
  // strided tiles put consecutive columns on consecutive lanes (always
  // coalesced); contiguous tiles put consecutive offsets j < S on
  // consecutive lanes, which gives >= 16-element runs when S >= 16.
  auto coalesced = [&](const OpDesc& op) { return s.mode == MODE_STRIDED || op.S >= 16; };
  const int io = env_int("PAFC_TUNE_IO", 13);
  const bool ld = s.mode == MODE_STRIDED ? (io & 4) : (io & 1);
  const bool st = s.mode == MODE_STRIDED ? (io & 8) : (io & 2);
  ops.front().src_g = (ld && !ops.front().cross && coalesced(ops.front())) ? 1 : 0;
  ops.back().dst_g = (st && !ops.back().cross && coalesced(ops.back())) ? 1 : 0;
  a.nops = (uint32_t)ops.size();
  for (size_t i = 0; i < ops.size(); ++i) a.ops[i] = ops[i];
  return true;
}

// Host-side bounds check of a pass descriptor, with the kernels' own index
// formulas: every tile touches positions i < L of valid columns c at
// base + i*S_i + c*S_c (base = o*S_o + col0*S_c); every op reads and writes
// positions b*K + j + s*S < L; twiddle indices stay below n_tw.  `extent` is
// the number of elements of the array (and of the filter spectrum) the pass
// runs over.
bool validate_pass(const PassArgs& a, int64_t extent, int64_t n_tw) {
  if (a.L == 0 || a.W == 0 || (a.W & (a.W - 1)) != 0 || a.LW != a.L * a.W) return false;
  if (a.tiles_per_slice != (a.ncols + a.W - 1) / a.W) return false;
  if (a.ntiles % a.tiles_per_slice != 0) return false;
  const int64_t nouter = a.ntiles / a.tiles_per_slice;
  const int64_t last_col = (int64_t)a.ncols - 1;
  const int64_t maxidx = (nouter - 1) * a.S_o + last_col * a.S_c + (int64_t)(a.L - 1) * a.S_i;
  if (maxidx >= extent || a.S_i <= 0 || a.S_c <= 0 || a.S_o < 0) return false;
  if (a.nops == 0 || a.nops > (uint32_t)kMaxOps) return false;
  // LDS twiddle tables: lo has 2^b entries, hi covers every exponent < n_tw,
  // and the flat source table is read at e << b < n_tw only
  if (!a.twl_global) {
    if (((int64_t)a.twl_nhi << a.twl_bits) < n_tw || (((int64_t)a.twl_nhi - 1) << a.twl_bits) >= n_tw)
      return false;
    if (((int64_t)1 << a.twl_bits) > n_tw && n_tw > 1) return false;
  }
  uint32_t K = a.L;
  for (uint32_t k = 0; k < a.nops; ++k) {
    const OpDesc& op = a.ops[k];
    if (op.cross) {  // legs hi*R*cs + p*cs + lo < W of one full tile row
      if (a.mode != MODE_STRIDED || a.W != a.ncols || a.tiles_per_slice != 1) return false;
      if (op.R < 2 || op.tw || op.src_g || op.dst_g || op.cs == 0) return false;
      if (a.W % ((uint32_t)op.R * op.cs) != 0 || op.divCs.d != op.cs) return false;
      if (op.divQ.d != a.W / (uint32_t)op.R || op.nitems != a.L * (a.W / (uint32_t)op.R)) return false;
      if (op.type == OP_MID) return false;
      continue;
    }
    if (op.K == 0 || op.R < 2 || op.S * (uint32_t)op.R != op.K || a.L % op.K != 0) return false;
    if (op.nitems != (a.L / (uint32_t)op.R) * a.W) return false;
    if (op.Kf != op.K * a.jmul || (int64_t)op.Kf * op.escale != n_tw) return false;
    if (op.divS.d != op.S || op.divNB.d != a.L / op.K) return false;
    if (op.type == OP_MID && op.S != 1) return false;
    if (a.col_in_j && (uint64_t)a.jmul * a.divJc.d != a.ncols) return false;
    (void)K;
  }
  return true;
}

// The pipelined kernel runs a piece whose register groups are all the same
// (r, g), one item per thread: with flat twiddles of the piece's own length,
// or (*outer) a strided outer piece of a cut axis with the whole axis's
// twiddles from a two-level LDS copy, or from the global table when the copy
// would not fit (PAFC_PIPE_OUTER=0: general engine).
// Any pass (when gm and xc are asked for) may also have an innermost group
// of fewer stages (*gm < *g; its op runs R / r^gm groups per thread) and, in
// a strided tile whose row is exactly the folded faster axes, up to two
// folded axes of length 2 (*xc; their DFTs are exchanged across lanes) --
// PAFC_PIPE_MIDX=0 turns both off.
bool pipe_shape(const Seg& s, const std::vector<CrossAxis>* cross, int* r, int* g, int* ng,
                bool* outer = nullptr, int kind = -1, int* gm = nullptr, int* xc = nullptr) {
  if (gm) *gm = -1;
  if (xc) *xc = 0;
  if (env_int("PAFC_PIPE", 1) == 0) return false;
  const bool out = s.col_in_j != 0 && s.mode == MODE_STRIDED;
  // a piece without an LDS twiddle copy runs pipelined only as an outer
  // piece (which reads the global table and forms the powers itself)
  if (s.tw_global && !out) return false;
  if (out ? env_int("PAFC_PIPE_OUTER", 1) == 0 : (s.jmul != 1 || s.n_tw != (int64_t)s.L))
    return false;
  const bool ext = kind >= 0 && !out && gm && xc && env_int("PAFC_PIPE_MIDX", 1) != 0;
  int ncross = 0;
  if (cross && !cross->empty()) {
    if (!ext || s.mode != MODE_STRIDED || cross->size() > 2) return false;
    for (const CrossAxis& c : *cross)
      if (c.r != 2 || c.g != 1 || c.cs != (1u << ncross++)) return false;
    if (s.W != (1u << ncross) || s.ncols != s.W) return false;
  }
  const auto groups = group_runs(s.rho, s.caps);
  if (groups.empty()) return false;
  for (size_t i = 0; i + 1 < groups.size(); ++i)
    if (groups[i] != groups[0]) return false;
  const auto& last = groups.back();  // the innermost group (DIF order)
  if (last.first != groups[0].first || last.second > groups[0].second) return false;
  const bool uniform = last == groups[0] && ncross == 0;
  if (!uniform && !ext) return false;
  *r = groups[0].first;
  *g = groups[0].second;
  *ng = (int)groups.size();
  if (outer) *outer = out;
  if (uniform) return out ? pipe_outer_supported(*r, *g, *ng) : pipe_supported(*r, *g, *ng);
  *gm = last.second;
  *xc = ncross;
  return pipe_ext_supported(*r, *g, *ng, *gm, *xc, kind, (int)s.mode);
}

bool make_pass(const Seg& s_in, int kind, size_t elem, Pass* p,
               const std::vector<CrossAxis>* cross = nullptr) {
  // a piece of short groups (R <= 9) can take one item per thread in blocks
  // of up to 1024 threads: narrow its tile until it holds that many items
  Seg s = s_in;
  {
    // odd-radix pieces run one thread per R-point item: narrow the tile
    // until its block holds them
    int r = 0, g = 0, ng = 0, gm = -1, xc = 0;
    if (pipe_shape(s, cross, &r, &g, &ng, nullptr, kind, &gm, &xc) && xc == 0 &&
        (r == 3 || r == 5)) {
      const uint32_t R = (uint32_t)ipow64(r, g);
      const uint32_t lim = (uint32_t)pipe_thread_limit(r, g, elem == 16, 0);
      while (s.W > 1 && (s.L / R) * s.W > lim) s.W /= 2;
    }
  }
  PassArgs& a = p->a;
  memset(&a, 0, sizeof(a));
  a.mode = s.mode;
  a.L = s.L;
  a.W = s.W;
  a.logW = ilog2u(s.W);
  a.LW = s.L * s.W;
  a.S_i = s.S_i;
  a.S_c = s.S_c;
  a.S_o = s.S_o;
  a.ncols = s.ncols;
  a.tiles_per_slice = (s.ncols + s.W - 1) / s.W;
  a.ntiles = a.tiles_per_slice * s.nouter;
  a.jmul = s.jmul;
  a.col_in_j = s.col_in_j;
  a.divL = make_fastdiv(s.L);
  a.divTiles = make_fastdiv(a.tiles_per_slice);
  a.divJc = make_fastdiv(s.jcdiv);
  a.lds_sh = s.mode == MODE_CONTIG && (s.L & 1u) && env_int("PAFC_LDS_PAD", 0) == 0 ? 31u : 4u;
  if (!build_ops(s, kind, a, &p->cls, cross)) return false;
  uint32_t maxitems = 0;
  for (uint32_t i = 0; i < a.nops; ++i) maxitems = std::max(maxitems, a.ops[i].nitems);
  uint32_t th = std::min<uint32_t>(kMaxThreads, ((maxitems + 63) / 64) * 64);
  p->threads = std::max<uint32_t>(64, th);
  // LDS copy of the twiddles, two-level with ~sqrt(n_tw) entries per level
  // (the same split rule as the global table when that one is two-level),
  // unless the piece reads the global table
  a.twl_global = s.tw_global ? 1u : 0u;
  {
    uint32_t b = 0;
    while (((int64_t)1 << (2 * b)) < s.n_tw) ++b;
    a.twl_bits = b;
    a.twl_nhi = (uint32_t)((s.n_tw + ((int64_t)1 << b) - 1) >> b);
    const uint64_t LW = a.LW;
    a.twl_off = (uint32_t)((LW + (LW >> 4) + 2) & ~1ull);
  }
  p->lds = (size_t)(a.twl_off + (s.tw_global ? 0u : (1u << a.twl_bits) + a.twl_nhi)) * elem;
  if (p->lds > s.lds) return false;
  p->tw_n = s.n_tw;
  p->mid = (kind == 2);
  p->kind = 0;
  // pipelined kernel: every group of the piece has the same (r, g), each op
  // has one item per thread, flat twiddles of the piece's own length
  {
    int r = 0, g = 0, ng = 0, gm = -1, xc = 0;
    bool outer = false;
    // it also addresses with 32-bit byte offsets: the span of elements the
    // pass touches must stay below 4 GiB
    const uint64_t span = (uint64_t)(s.nouter - 1) * (uint64_t)s.S_o +
                          (uint64_t)(s.L - 1) * (uint64_t)s.S_i +
                          (uint64_t)(s.ncols - 1) * (uint64_t)s.S_c + 1;
    bool ok = pipe_shape(s, cross, &r, &g, &ng, &outer, kind, &gm, &xc) &&
              span * elem <= 0xFFFFFFFFull;
    // a middle pass with a short innermost group or folded columns
    const bool ext = ok && gm >= 0;
    // an outer piece is never the middle pass (the product sits in the
    // innermost piece)
    if (outer && kind == 2) ok = false;
    // the kernel takes each op's twiddle scale from the descriptor by its
    // own op index, so the two op orders must agree (forward: K = L / R^i,
    // inverse: K = R^(i+1)), every op with twiddles
    if (ok && outer) {
      const uint32_t R = (uint32_t)ipow64(r, g);
      uint32_t Kd = s.L, Ku = R;
      for (uint32_t i = 0; ok && i < a.nops; ++i, Kd /= R, Ku *= R)
        ok = a.ops[i].K == (kind == 0 ? Kd : Ku) && a.ops[i].tw == 1;
    }
    // one item per thread: the radix-16 shapes in whole waves (as the
    // general engine would size the block), the short ones in blocks of
    // exactly one thread per item
    uint32_t items = a.nops ? a.ops[0].nitems : 0;
    if (ext) {
      // one R-point item per thread in every op: the innermost group's op
      // (last forward, first inverse, the middle op) runs R / RM groups of
      // RM points; the column ops run inside the first and last op
      const uint32_t R = (uint32_t)ipow64(r, g), RM = (uint32_t)ipow64(r, gm);
      items = a.LW / R;
      std::vector<uint32_t> want;  // group sizes of the axis ops, in op order
      for (int q = 0; q < ng - 1 && kind != 1; ++q) want.push_back(R);
      want.push_back(RM);
      for (int q = 0; q < ng - 1 && kind != 0; ++q) want.push_back(R);
      size_t n = 0;
      for (uint32_t i = 0; ok && i < a.nops; ++i) {
        const OpDesc& o = a.ops[i];
        if (o.cross) continue;
        ok = n < want.size() && (uint32_t)o.R == want[n] &&
             (o.R != (int32_t)RM || o.R == (int32_t)R || o.nitems == a.LW / RM) &&
             (o.R != (int32_t)R || o.nitems == items);
        ++n;
      }
      ok = ok && n == want.size();
      // (folded columns exchange values across lanes: whole waves)
      ok = ok && (xc == 0 || items % 64 == 0) &&
           items <= (uint32_t)pipe_thread_limit(r, g, elem == 16, xc);
    } else {
      for (uint32_t i = 0; ok && i < a.nops; ++i) ok = a.ops[i].nitems == items;
    }
    // odd radices: one thread per item, any count within the block limit
    const bool small = ok && !ext && (r == 3 || r == 5);
    // (4096-long axes in four radix-8 groups: one 512-thread block, where
    // the general engine's count is decided below)
    if (ok && !ext)
      ok = small ? items <= (uint32_t)pipe_thread_limit(r, g)
                 : items == p->threads ||
                       (((ipow64(r, g) == 8 && ng == 4) || (ipow64(r, g) == 4 && ng == 6)) &&
                        items > p->threads &&
                        items <= (uint32_t)pipe_uniform_threads(r, g, ng));
    if (ok) {
      p->pipe = true;
      p->pipe_r = r;
      p->pipe_g = g;
      p->pipe_ng = ng;
      p->pipe_kind = kind;
      p->pipe_mode = outer ? (int)MODE_OUTER : (int)s.mode;
      p->pipe_gm = ext ? gm : g;
      p->pipe_xc = ext ? xc : 0;
      p->pipe_threads = items;
      const uint64_t LW = a.LW;
      // tile, then the flat table of the piece (or, outer, the two-level
      // table of the general engine's layout)
      // (long contiguous or column-folded tiles of even length pad the table
      // one in 16, as the kernel's pipe_tw_pad)
      const bool twpad = (s.mode == MODE_CONTIG || (ext && xc > 0)) && s.L % 2 == 0 && s.L >= 1024;
      p->pipe_lds = outer ? p->lds
                          : (size_t)(((LW + (LW >> 4) + 2) & ~1ull) + s.L + (twpad ? s.L / 16 : 0)) *
                                elem;
    }
  }
  // wide register class: every group R <= 9 and every op at least two full
  // rounds of a 256-thread block -> (nearly) one item per thread, up to 1024
  // threads.  Ops with fewer items would leave most of a wide block idle and
  // cost resident blocks (measured slower), so they stay in the small class.
  // (Decided for pipelined passes too: the general engine is their fallback.)
  {
    int maxR = 0;
    uint32_t maxitems = 0, minitems = UINT32_MAX;
    for (uint32_t i = 0; i < a.nops; ++i) {
      maxR = std::max(maxR, (int)a.ops[i].R);
      maxitems = std::max(maxitems, a.ops[i].nitems);
      minitems = std::min(minitems, a.ops[i].nitems);
    }
    if (maxR <= 9 && minitems >= 2 * kMaxThreads && env_int("PAFC_WIDE", 1) != 0) {
      p->cls = 2;
      p->threads = std::min<uint32_t>(kMaxWideThreads, ((maxitems + 63) / 64) * 64);
    }
  }
  char buf[160];
  std::string ops;
  for (uint32_t i = 0; i < a.nops; ++i) {
    const OpDesc& o = a.ops[i];
    snprintf(buf, sizeof(buf), "%s%s%s%d", i ? "," : "", o.cross ? "X" : "",
             o.type == OP_DIF ? "DIF" : o.type == OP_DIT ? "DIT" : "MID", o.R);
    ops += buf;
  }
  snprintf(buf, sizeof(buf), "%s L=%u W=%u tiles=%u thr=%u [", s.mode == MODE_STRIDED ? "strided" : "contig",
           s.L, s.W, a.ntiles, p->pipe ? p->pipe_threads : p->threads);
  p->label = std::string(buf) + ops + "]";
  if (s.tw_global) p->label += " twg";

  if (p->pipe) {
    char nm[96];
    if (p->pipe_gm != p->pipe_g || p->pipe_xc != 0)
      snprintf(nm, sizeof(nm), " pipe_kernel<%s,%d,%d,%d,%d,%d,%d,%d>",
               elem == 16 ? "double" : "float", p->pipe_r, p->pipe_g, p->pipe_ng, kind,
               p->pipe_mode, p->pipe_gm, p->pipe_xc);
    else
      snprintf(nm, sizeof(nm), " pipe_kernel<%s,%d,%d,%d,%d,%d>", elem == 16 ? "double" : "float",
               p->pipe_r, p->pipe_g, p->pipe_ng, kind, p->pipe_mode);
    p->label += nm;
  }
  return true;
}

// Pieces of one (sub-)axis of length n (stages rho, innermost first) at
// element stride st, repeated over `outer` blocks spaced n*st apart.  Appends
// the pieces outermost first; false if some piece cannot fit LDS.
bool split_axis(int64_t n, const std::vector<int>& rho, int64_t st, int64_t outer, size_t elem,
                const GroupCaps& caps, const TuneVal* tv, const TuneVal* tsplit,
                std::vector<Seg>& segs, size_t budget) {
  const int t = (int)rho.size();
  // LDS of a strided piece's tile (16 columns, or the stride) above which
  // the axis is cut: one resident block per CU otherwise
  const size_t strided_cap = (size_t)std::max(8, env_int("PAFC_TUNE_STRIDED_KB", 72)) * 1024;
  auto tile16 = [&](int64_t L) { return tile_lds_bytes((uint64_t)L * 16, elem); };
  // a strided piece's tile is at most 16 columns wide, and no wider than
  // the stride (its column count)
  const uint64_t wcap = pow2_floor((uint64_t)std::min<int64_t>(st, 16));
  auto tilew = [&](int64_t L) { return tile_lds_bytes((uint64_t)L * wcap, elem); };
  int ti = 0;
  int64_t ni = 1;
  if (tsplit) {
    while (ti < t && ni < tsplit->split) ni *= rho[ti++];
    if (ni != tsplit->split) return false;
  } else if (!fits_lds(n, elem, budget) && st == 1) {
    const size_t cap = elem == 16 ? 4096 : 8192;
    while (ti < t - 1 && ni * rho[ti] <= (int64_t)cap) ni *= rho[ti++];
  } else if (st > 1 && tilew(n) > strided_cap) {
    while (ti < t - 1 && tilew(ni * rho[ti]) <= strided_cap) ni *= rho[ti++];
    if (n / ni < 2) ti = 0, ni = 1;
  }
  // an outer piece that does not fit LDS, or whose tile would be too narrow
  // (short row segments), takes fewer stages: the inner length grows, and is
  // cut again below
  auto outer_width = [&](int64_t L) {
    Seg o;
    o.mode = MODE_STRIDED;
    o.L = (uint32_t)L;
    o.ncols = (uint32_t)std::min<int64_t>(n / L * st, UINT32_MAX);
    o.n_tw = n;
    o.lds = budget;
    o.tw_global = twiddles_global(L, n, elem, budget);
    choose_width(o, elem, 0);
    return o.W;
  };
  if (ti > 0 && !tsplit) {
    if (!fits_lds(n / ni, elem, budget)) {
      // far too long for one outer piece: 16-column outer tiles within
      // 72 KB, like every other strided pass
      while (ti < t - 1 && tile16(n / ni) > strided_cap) ni *= rho[ti++];
    } else {
      // 8 columns at least; an axis of a grid (stride > 1) is held to the
      // 16-column tiles within 72 KB of every other strided pass (the 1-D
      // pieces keep 8 columns: the tuned 1-D plans were measured so)
      while (ti < t - 1 &&
             (outer_width(n / ni) < 8 || (st > 1 && tile16(n / ni) > strided_cap)))
        ni *= rho[ti++];
    }
  }
  if (ti == 0) {
    if (!fits_lds(n, elem, budget)) return false;
    Seg s;
    s.L = (uint32_t)n;
    s.rho = rho;
    s.n_tw = n;
    s.caps = caps;
    if (st == 1) {
      s.mode = MODE_CONTIG;
      s.S_i = 1;
      s.S_c = n;
      s.ncols = (uint32_t)outer;
      s.S_o = 0;
      s.nouter = 1;
    } else {
      s.mode = MODE_STRIDED;
      s.S_i = st;
      s.S_c = 1;
      s.ncols = (uint32_t)st;
      s.S_o = n * st;
      s.nouter = (uint32_t)outer;
    }
    if ((uint64_t)outer >= (1ull << 32) || (uint64_t)st >= (1ull << 32)) return false;
    s.lds = budget;
    s.tw_global = twiddles_global(s.L, s.n_tw, elem, budget);
    choose_width(s, elem, tv ? tv->W : 0);
    if (tile_lds_bytes(s.L * (uint64_t)s.W, elem) > budget) return false;
    segs.push_back(s);
    return true;
  }
  const int64_t no = n / ni;
  if (!fits_lds(no, elem, budget) || ti == t) return false;
  if ((uint64_t)ni * st >= (1ull << 32) || (uint64_t)outer * no >= (1ull << 32)) return false;
  // element (o, i_o, i_i, f) of the sub-axis sits at
  // o*n*st + i_o*ni*st + i_i*st + f
  Seg so;  // outer: positions i_o < no at stride ni*st, columns (i_i, f)
  so.mode = MODE_STRIDED;
  so.L = (uint32_t)no;
  so.S_i = ni * st;
  so.S_c = 1;
  so.ncols = (uint32_t)(ni * st);
  so.S_o = n * st;
  so.nouter = (uint32_t)outer;
  so.jmul = (uint32_t)ni;
  so.col_in_j = 1;
  so.jcdiv = (uint32_t)st;
  so.n_tw = n;
  so.rho.assign(rho.begin() + ti, rho.end());
  so.caps = caps;
  so.lds = budget;
  so.tw_global = twiddles_global(so.L, so.n_tw, elem, budget);
  choose_width(so, elem, tv ? tv->Wo : 0);
  segs.push_back(so);
  // inner: an axis of length ni at stride st, one block per (o, i_o); its
  // radix-3 grouping may be tuned apart from the outer piece's
  const std::vector<int> rin(rho.begin(), rho.begin() + ti);
  GroupCaps caps_in = caps;
  if (tv && tv->gmax3i > 0) caps_in.g3 = std::min(tv->gmax3i, caps.lim3 > 0 ? caps.lim3 : 3);
  return split_axis(ni, rin, st, outer * no, elem, caps_in, tv, nullptr, segs, budget);
}

// Limits a caller may put on a plan beyond the device's: the LDS one tile
// may use, and the largest radix-3 / radix-5 register groups (0: no limit
// beyond the planner's own).  The persistent batched launch runs every pass
// of every size class in one kernel whose LDS size and register class are
// fixed for the whole launch.
struct PlanLimits {
  size_t lds = kLdsBudget;
  int g3 = 0, g5 = 0;
  bool table = true;  // take the tuning table's entries
  bool batched = false;  // a size class of the batched form
};

pafc_status plan_once(PlanCore& P, int ndim, const int64_t* dims, const int* radix, int dtype,
                      int variant, bool use_table, const PlanLimits& lim) {
  if (ndim < 1 || ndim > 3 || !dims) return PAFC_ERROR_INVALID_VALUE;
  if (dtype != PAFC_C64 && dtype != PAFC_C128) return PAFC_ERROR_INVALID_VALUE;
  if (variant < PAFC_PERM_FREE || variant > PAFC_PERM_FREE_UNFUSED) return PAFC_ERROR_INVALID_VALUE;
  P.ndim = ndim;
  P.dtype = dtype;
  P.variant = variant;
  P.elem = dtype == PAFC_C128 ? 16 : 8;
  P.N = 1;
  for (int a = 0; a < ndim; ++a) {
    if (dims[a] < 2) return PAFC_ERROR_INVALID_VALUE;
    if (dims[a] > (int64_t)1 << 30) return PAFC_ERROR_UNSUPPORTED_SIZE;
    P.dims[a] = dims[a];
    P.N *= dims[a];
  }
  if (P.N > ((int64_t)1 << 34)) return PAFC_ERROR_UNSUPPORTED_SIZE;
  P.axes.resize(ndim);
  for (int a = 0; a < ndim; ++a) {
    AxisInfo& ax = P.axes[a];
    ax.n = dims[a];
    int r = radix ? radix[a] : 0;
    if (r == 0) {
      if (!auto_rho(ax.n, &ax.rho)) return PAFC_ERROR_UNSUPPORTED_SIZE;
    } else {
      if (r != 2 && r != 3 && r != 4 && r != 5 && r != 8) return PAFC_ERROR_UNSUPPORTED_SIZE;
      int64_t m = ax.n;
      int t = 0;
      while (m % r == 0) { m /= r; ++t; }
      if (m != 1) return PAFC_ERROR_UNSUPPORTED_SIZE;
      ax.rho.assign(t, r);
    }
    ax.pos = pos_table(ax.n, ax.rho);
    ax.posinv.assign((size_t)ax.n, 0);
    for (int64_t k = 0; k < ax.n; ++k) ax.posinv[(size_t)ax.pos[(size_t)k]] = (int32_t)k;
  }
  // Segments: every axis is one pass unless it is cut into pieces (below).
  for (int a = 0; a < ndim; ++a) {
    AxisInfo& ax = P.axes[a];
    int64_t st = 1, outer = 1;
    for (int b = a + 1; b < ndim; ++b) st *= dims[b];
    for (int b = 0; b < a; ++b) outer *= dims[b];
    TuneVal tv;
    bool tuned = use_table && tune_lookup(dtype, ax.n, &tv);
    GroupCaps caps;
    caps.g3 = tuned && tv.gmax3 > 0 ? tv.gmax3 : env_int("PAFC_TUNE_GMAX3", 3);
    caps.g5 = tuned && tv.gmax5 > 0 ? tv.gmax5 : env_int("PAFC_TUNE_GMAX5", 2);
    if (lim.g3 > 0) caps.g3 = std::min(caps.g3, lim.g3);
    caps.lim3 = lim.g3;
    if (lim.g5 > 0) caps.g5 = std::min(caps.g5, lim.g5);
    // A 1-D transform of 4096 radix-2 stages is one tile: four groups of
    // 2^3 in a 512-thread block run it faster than three of 2^4 in 256
    // threads (more waves to cover the LDS round trips, fewer registers)
    const bool single4096 = ndim == 1 && ax.n == 4096 && !lim.batched;
    caps.g2 = single4096 && ax.rho.size() == 12 && ax.rho[0] == 2
                  ? env_int("PAFC_TUNE_GMAX2_4096", 3)
                  : 4;
    // and in FP32 (not FP64, measured 1 % slower) six groups of radix 4 in a
    // 1024-thread block run a 1-D 4096-point radix-4 transform faster than
    // three of 4^2 in 256 threads.  Not in the batched form, whose size
    // classes fill the device with many such problems at once (measured
    // 1-2 % slower there).
    caps.g4 = single4096 && ax.rho.size() == 6 && ax.rho[0] == 4
                  ? env_int("PAFC_TUNE_GMAX4_4096", dtype == PAFC_C64 ? 1 : 2)
                  : 2;
    // Cut the axis into pieces (G2): an outer piece takes its outermost
    // stages, strided over the inner length; the inner length is again an
    // axis of its own and is cut the same way while it is too long.  A piece
    // is cut when its whole-axis tile does not fit LDS (contiguous), when a
    // strided tile 16 columns wide would leave the CU with a single resident
    // block, or at the top level of a 1-D transform when the tuning table
    // says so (the table is measured on 1-D transforms).
    const TuneVal* tvp = tuned && tv.split > 0 && tv.split < ax.n && ndim == 1 ? &tv : nullptr;
    if (!split_axis(ax.n, ax.rho, st, outer, P.elem, caps, tuned ? &tv : nullptr, tvp, ax.segs,
                    lim.lds))
      return PAFC_ERROR_UNSUPPORTED_SIZE;
  }
  // twiddle tables, one per distinct n_tw
  for (auto& ax : P.axes)
    for (auto& s : ax.segs) {
      if (P.tw.count(s.n_tw)) continue;
      TwTable t;
      t.n = s.n_tw;
      t.lo_off = P.tw_elems;
      if (s.n_tw <= 16384) {
        P.tw_elems += s.n_tw;
      } else {
        uint32_t bits = 0;
        while (((int64_t)1 << (2 * bits)) < s.n_tw) ++bits;
        t.bits = bits;
        const int64_t nlo = (int64_t)1 << bits;
        const int64_t nhi = (s.n_tw + nlo - 1) >> bits;
        P.tw_elems += nlo;
        t.hi_off = P.tw_elems;
        P.tw_elems += nhi;
      }
      P.tw[s.n_tw] = t;
    }
  // pass sequences
  // the axis whose last piece carries the fused product: by default the
  // slowest axis, so its (most strided) pass is touched once
  const int mid = std::min(ndim - 1, std::max(0, env_int("PAFC_TUNE_MID", 0)));
  P.middle = mid;
  auto add = [&](std::vector<Pass>& v, const Seg& s, int kind) -> bool {
    Pass p;
    if (!make_pass(s, kind, P.elem, &p)) return false;
    v.push_back(p);
    return true;
  };
  // Short faster axes folded into a pass of the slowest axis as column ops:
  // its innermost piece is strided over all the other axes; when each of
  // them is one register group and together they form a tile row of at
  // most 64 power-of-two columns, the tile holds whole rows and their DFTs
  // run inside that pass -- the fused middle pass of the permutation-free
  // convolution, and the innermost forward and inverse passes of the
  // slowest axis in the transforms alone (the anisotropic grids n x 2,
  // n x 2 x 2 then move 5 and 5 passes instead of 7 and 9).
  std::vector<CrossAxis> fold;
  Seg mseg = P.axes[mid].segs.back();
  if (mid == 0 && ndim > 1 && env_int("PAFC_FOLD", 1) != 0) {
    bool ok = mseg.mode == MODE_STRIDED;
    int64_t cs = 1;
    for (int a = ndim - 1; a >= 1 && ok; --a) {
      const AxisInfo& ax = P.axes[a];
      const auto groups = group_runs(ax.rho, ax.segs[0].caps);
      ok = ax.segs.size() == 1 && groups.size() == 1;
      if (ok) fold.push_back(CrossAxis{groups[0].first, groups[0].second, (uint32_t)cs});
      cs *= ax.n;
    }
    ok = ok && cs == (int64_t)mseg.ncols && (cs & (cs - 1)) == 0 && cs <= 64;
    if (ok) {
      mseg.W = (uint32_t)cs;
      const size_t tw = mseg.tw_global ? 0 : twl_bytes(mseg.n_tw, P.elem);
      ok = tile_lds_bytes((uint64_t)mseg.L * mseg.W, P.elem) + tw <= lim.lds;
    }
    if (!ok) fold.clear();
  }
  auto add_folded = [&](std::vector<Pass>& v, int kind) -> bool {
    Pass p;
    if (!make_pass(mseg, kind, P.elem, &p, &fold)) return false;
    v.push_back(p);
    return true;
  };
  // forward only: all axes, fastest first, outer piece before inner piece
  // (folded: the slowest axis alone, its innermost piece with the others)
  const auto& s0 = P.axes[0].segs;
  for (int a = ndim - 1; a >= 0; --a) {
    if (!fold.empty() && a != 0) continue;
    for (size_t i = 0; i < P.axes[a].segs.size(); ++i) {
      const bool f = !fold.empty() && i + 1 == s0.size();
      if (!(f ? add_folded(P.fwd, 0) : add(P.fwd, P.axes[a].segs[i], 0)))
        return PAFC_ERROR_UNSUPPORTED_SIZE;
    }
  }
  // inverse only: the mirror image
  for (int a = 0; a < ndim; ++a) {
    if (!fold.empty() && a != 0) continue;
    for (size_t i = P.axes[a].segs.size(); i-- > 0;) {
      const bool f = !fold.empty() && i + 1 == s0.size();
      if (!(f ? add_folded(P.inv, 1) : add(P.inv, P.axes[a].segs[i], 1)))
        return PAFC_ERROR_UNSUPPORTED_SIZE;
    }
  }
  if (variant == PAFC_PERM_FREE) {
    // the other axes' forward passes, fastest axis first (PAFC_AXIS_ORDER=1:
    // slowest first), their inverse passes in the mirrored order
    std::vector<int> order;
    for (int a = ndim - 1; a >= 0; --a)
      if (a != mid && fold.empty()) order.push_back(a);
    if (env_int("PAFC_AXIS_ORDER", 0) == 1) std::reverse(order.begin(), order.end());
    for (int a : order)
      for (auto& s : P.axes[a].segs)
        if (!add(P.conv, s, 0)) return PAFC_ERROR_UNSUPPORTED_SIZE;
    auto& ms = P.axes[mid].segs;
    for (size_t i = 0; i + 1 < ms.size(); ++i)
      if (!add(P.conv, ms[i], 0)) return PAFC_ERROR_UNSUPPORTED_SIZE;
    if (fold.empty()) {
      if (!add(P.conv, ms.back(), 2)) return PAFC_ERROR_UNSUPPORTED_SIZE;
    } else {
      Pass p;
      if (!make_pass(mseg, 2, P.elem, &p, &fold)) return PAFC_ERROR_UNSUPPORTED_SIZE;
      P.conv.push_back(p);
    }
    for (size_t i = ms.size() - 1; i-- > 0;)
      if (!add(P.conv, ms[i], 1)) return PAFC_ERROR_UNSUPPORTED_SIZE;
    for (auto a = order.rbegin(); a != order.rend(); ++a)
      for (auto it = P.axes[*a].segs.rbegin(); it != P.axes[*a].segs.rend(); ++it)
        if (!add(P.conv, *it, 1)) return PAFC_ERROR_UNSUPPORTED_SIZE;
  } else {
    for (auto& p : P.fwd) P.conv.push_back(p);
    if (variant == PAFC_PERM_FREE_UNFUSED) {
      Pass m;
      m.kind = 1;
      m.label = "mul";
      P.conv.push_back(m);
    } else {
      Pass p1;
      p1.kind = 2;
      p1.perm_dir = 1;
      p1.label = "permute dr->nat x H";
      Pass p2;
      p2.kind = 2;
      p2.perm_dir = 2;
      p2.label = "permute nat->dr";
      P.conv.push_back(p1);
      P.conv.push_back(p2);
    }
    for (auto& p : P.inv) P.conv.push_back(p);
  }
  for (auto* seq : {&P.conv, &P.fwd, &P.inv})
    for (const Pass& ps : *seq)
      if (ps.kind == 0 && !validate_pass(ps.a, P.N, ps.tw_n)) return PAFC_ERROR_UNSUPPORTED_SIZE;
  // algorithmic HBM bytes: each pass reads and writes N elements once; the
  // product reads the spectrum once more
  auto bytes = [&](const std::vector<Pass>& v) {
    int64_t b = 0;
    const int64_t ne = P.N * (int64_t)P.elem;
    for (auto& p : v) {
      if (p.kind == 0) b += 2 * ne + (p.mid ? ne : 0);
      else if (p.kind == 1) b += 3 * ne;
      else if (p.kind == 2) b += 2 * ne + (p.perm_dir == 1 ? ne : 0);
    }
    return b;
  };
  P.hbm_conv = bytes(P.conv);
  P.hbm_fwd = bytes(P.fwd);
  return PAFC_SUCCESS;
}

// A tuning entry is keyed by axis length alone, so a choice measured for an
// axis of one shape can be infeasible for the same length in another (the
// 2187 axis of a 2187 x 2187 grid is cut into pieces, a 2187-point 1-D
// transform is one middle pass, which single radix-3 groups would give more
// ops than a pass holds): the plan is then made with the planner defaults.
pafc_status plan_core(PlanCore& P, int ndim, const int64_t* dims, const int* radix, int dtype,
                      int variant, const PlanLimits& lim = PlanLimits()) {
  pafc_status st = plan_once(P, ndim, dims, radix, dtype, variant, lim.table, lim);
  if (st != PAFC_ERROR_UNSUPPORTED_SIZE) return st;
  P = PlanCore();
  return plan_once(P, ndim, dims, radix, dtype, variant, false, lim);
}

std::string describe_core(const PlanCore& P) {
  std::string s = "{";
  char b[256];
  snprintf(b, sizeof(b), "\"ndim\": %d, \"dims\": [", P.ndim);
  s += b;
  for (int a = 0; a < P.ndim; ++a) {
    snprintf(b, sizeof(b), "%s%lld", a ? ", " : "", (long long)P.dims[a]);
    s += b;
  }
  snprintf(b, sizeof(b), "], \"dtype\": \"%s\", \"variant\": %d, \"middle_axis\": %d, \"axes\": [",
           P.dtype == PAFC_C128 ? "c128" : "c64", P.variant, P.middle);
  s += b;
  for (int a = 0; a < P.ndim; ++a) {
    const AxisInfo& ax = P.axes[a];
    s += a ? ", {" : "{";
    snprintf(b, sizeof(b), "\"n\": %lld, \"rho\": [", (long long)ax.n);
    s += b;
    for (size_t i = 0; i < ax.rho.size(); ++i) {
      snprintf(b, sizeof(b), "%s%d", i ? ", " : "", ax.rho[i]);
      s += b;
    }
    s += "], \"pieces\": [";
    for (size_t i = 0; i < ax.segs.size(); ++i) {
      const Seg& g = ax.segs[i];
      snprintf(b, sizeof(b), "%s{\"L\": %u, \"W\": %u, \"mode\": \"%s\"}", i ? ", " : "", g.L, g.W,
               g.mode == MODE_STRIDED ? "strided" : "contig");
      s += b;
    }
    s += "]}";
  }
  s += "], \"conv_passes\": [";
  for (size_t i = 0; i < P.conv.size(); ++i) {
    s += i ? ", \"" : "\"";
    s += P.conv[i].label + "\"";
  }
  snprintf(b, sizeof(b), "], \"hbm_bytes_conv\": %lld, \"hbm_bytes_forward\": %lld, \"N\": %lld}",
           (long long)P.hbm_conv, (long long)P.hbm_fwd, (long long)P.N);
  s += b;
  return s;
}

}  // namespace

// ===================================================================== plan

struct pafc_plan_s {
  PlanCore P;
  int device = 0;
  void* d_tw = nullptr;
  void* d_H = nullptr;
  void* d_scratch = nullptr;
  int32_t* d_maps = nullptr;  // per axis: pos, posinv
  void* d_symtab = nullptr;   // per-axis symbol tables (FP64 complex), 3 + sum n_i
  PassArgs* d_descs = nullptr;
  // prime-factor route: the grid plan, its factors N0 <= N1 <= N2 (N0 = 1
  // for two factors) and the gather tables (CRT input map, then the
  // output map of the spectrum), N0 + N1 + N2 entries each
  pafc_plan_s* inner = nullptr;
  uint32_t pfa_N[3] = {1, 1, 1};
  uint32_t pfa_uinv = 0;  // (N0 N1)^-1 mod N2, for the tiled CRT map
  uint32_t* d_pfa_tab = nullptr;
  // Bluestein route (blue_m > 0): the inner plan has length blue_m; chirp
  // c_j (n entries) and the filter's natural-order spectrum (n entries)
  int64_t blue_m = 0;
  void* d_chirp = nullptr;
  void* d_hn = nullptr;
  // Rader route (rader_g > 0, the generator): the inner plan has length
  // n - 1; d_hn holds the spectrum in generator order (n entries);
  // d_rader_tab the powers g^m (n - 1 entries) then -log_g j (n entries);
  // d_rader_acc the block sums (kRaderBlocks x 4 doubles) then two constants
  int64_t rader_g = 0;
  uint32_t* d_rader_tab = nullptr;
  double* d_rader_acc = nullptr;
  std::vector<int64_t> map_off;
  // tile-major spectrum (PassArgs::h_tm): the middle pass of the convolution
  // and, in fwd_tm, the forward sequence whose last pass writes that order
  bool h_tm = false;
  // the comparison variants' product kernels read the spectrum streamed
  // (the arrays reach the last-level cache size)
  bool nt_h = false;
  int mid_pass = -1;  // index of the middle pass in P.conv
  std::vector<Pass> fwd_tm;
  bool filter_set = false;
  size_t bytes = 0;
  // pafc_convolve_with_filter_noalloc: this device's address of `scratch`
  // (NULL when the plan cannot use it, noalloc_status says why) and the
  // convolution sequence whose middle pass reads the spectrum from there
  void* noalloc_H = nullptr;
  pafc_status noalloc_status = PAFC_ERROR_INVALID_VALUE;
  std::vector<Pass> conv_noalloc;
};

namespace {

// Address of `scratch` on each device, looked up once per device with that
// device current (the first plan made on it), then reused.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

hipError_t scratch_address(int dev, void** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

pafc_status from_hip(hipError_t e) {
  if (e == hipSuccess) return PAFC_SUCCESS;
  if (e == hipErrorOutOfMemory) return PAFC_ERROR_OUT_OF_MEMORY;
  return PAFC_ERROR_DEVICE;
}

#define PAFC_TRY(expr)                         \
  do {                                         \
    pafc_status st_ = (expr);                  \
    if (st_ != PAFC_SUCCESS) return st_;       \
  } while (0)

// Events that only time launches: no system-scope fence (cache writeback
// and invalidate) when they are recorded, which would slow the launches they
// bracket; their times are read after a stream synchronisation.
hipError_t timing_event(hipEvent_t* e) {
  return hipEventCreateWithFlags(e, hipEventDisableSystemFence);
}

// Record event k of an event array, if there is an array and that entry
// exists (profiling runs may time a few launch positions only).
pafc_status rec(hipEvent_t* ev, size_t k, hipStream_t s) {
  if (!ev || !ev[k]) return PAFC_SUCCESS;
  return from_hip(hipEventRecord(ev[k], s));
}

bool aligned_for(const void* p, int dtype) {
  const uintptr_t m = dtype == PAFC_C128 ? 15 : 7;
  return ((uintptr_t)p & m) == 0;
}

void free_plan(pafc_plan_t p) {
  if (!p) return;
  if (p->d_tw) (void)hipFree(p->d_tw);
  if (p->d_H) (void)hipFree(p->d_H);
  if (p->d_scratch) (void)hipFree(p->d_scratch);
  if (p->d_maps) (void)hipFree(p->d_maps);
  if (p->d_symtab) (void)hipFree(p->d_symtab);
  if (p->d_descs) (void)hipFree(p->d_descs);
  if (p->d_pfa_tab) (void)hipFree(p->d_pfa_tab);
  if (p->d_chirp) (void)hipFree(p->d_chirp);
  if (p->d_hn) (void)hipFree(p->d_hn);
  if (p->d_rader_tab) (void)hipFree(p->d_rader_tab);
  if (p->d_rader_acc) (void)hipFree(p->d_rader_acc);
  if (p->inner) free_plan(p->inner);
  delete p;
}

const int32_t* map_ptr(pafc_plan_t p, int axis, bool inverse) {
  return p->d_maps + p->map_off[(size_t)axis] + (inverse ? p->P.axes[(size_t)axis].n : 0);
}

// Fill the device pointers of a pass descriptor (filter spectrum, twiddles).
void finalize_args(const PlanCore& P, const void* d_tw, const void* H, const Pass& ps,
                   PassArgs* a) {
  *a = ps.a;
  a->H = H;
  a->hscale = 1.0 / (double)P.N;  // the single 1/N, applied with the spectrum
  const TwTable& t = P.tw.at(ps.tw_n);
  const char* base = (const char*)d_tw;
  a->tw_lo = base + t.lo_off * (int64_t)P.elem;
  a->tw_hi = t.hi_off >= 0 ? base + t.hi_off * (int64_t)P.elem : nullptr;
  a->tw_bits = t.bits;
}

// Does this pass launch the pipelined kernel (whose launch can carry its own
// timing events)?
bool pass_binds_events(const Pass& ps) { return ps.kind == 0 && ps.pipe && ps.pipe_grid > 0; }

// Launch one kernel pass reading `in` and writing `out`.  t0 / t1 (only for
// a pass where pass_binds_events holds) take the launch's start and end.
pafc_status run_pass(pafc_plan_t p, const Pass& ps, const void* in, void* out, hipStream_t s,
                     hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr) {
  const bool dbl = p->P.dtype == PAFC_C128;
  if (ps.kind != 0) return PAFC_ERROR_INVALID_VALUE;
  if (ps.pipe && ps.pipe_grid > 0)
    return from_hip(launch_pipe(dbl, ps.pipe_r, ps.pipe_g, ps.pipe_ng, ps.pipe_kind, ps.pipe_mode,
                                p->d_descs + ps.desc, ps.pipe_grid, ps.pipe_threads, ps.pipe_lds,
                                in, out, s, ps.pipe_gm, ps.pipe_xc, t0, t1));
  if (t0 || t1) return PAFC_ERROR_INVALID_VALUE;

  return from_hip(launch_pass(dbl, ps.cls, p->d_descs + ps.desc, ps.a.ntiles, in, out, ps.threads,
                              ps.lds, s));
}

// Index-reversal permutation pass of the explicit variant:
// dir 1: out[k] = in[pos(k)] (* H / N),  dir 2: out[p] = in[posinv(p)].
pafc_status run_permute(pafc_plan_t p, int dir, const void* in, void* out, const void* h,
                        hipStream_t s) {
  const PlanCore& P = p->P;
  const double hs = 1.0 / (double)P.N;
  const bool dbl = P.dtype == PAFC_C128;
  const bool inv = dir == 2;
  const bool nt = h != nullptr && p->nt_h;
  uint32_t n0 = 1, n1 = 1, nl = (uint32_t)P.dims[P.ndim - 1];
  const int32_t* m0 = nullptr;
  const int32_t* m1 = nullptr;
  const int32_t* ml = map_ptr(p, P.ndim - 1, inv);
  if (P.ndim == 3) {
    n0 = (uint32_t)P.dims[0];
    n1 = (uint32_t)P.dims[1];
    m0 = map_ptr(p, 0, inv);
    m1 = map_ptr(p, 1, inv);
  } else if (P.ndim == 2) {
    n1 = (uint32_t)P.dims[0];
    m1 = map_ptr(p, 0, inv);
  }
  const bool pow2 = (nl & (nl - 1)) == 0;
  if (pow2 && nl <= 4096 && ((uint64_t)n0 * n1 * nl) % 4096 == 0) {
    const uint32_t log_nl = ilog2u(nl);
    return from_hip(launch_permute_tile(dbl, in, out, h, m0, m1, ml, n0, n1, log_nl, hs, nt, s));
  }
  if (tile_lds_bytes(nl, P.elem) <= kLdsBudget) {
    uint32_t rows = std::max<uint32_t>(1, 2048 / nl);
    while (rows > 1 && tile_lds_bytes((uint64_t)rows * nl, P.elem) > 64 * 1024) rows /= 2;
    return from_hip(launch_permute_rows(dbl, in, out, h, m0, m1, ml, n0, n1, nl, rows, hs, nt, s));
  }
  return from_hip(launch_permute_gather(dbl, in, out, h, m0, m1, ml, n0, n1, nl, hs, nt, s));
}

// Run a pass sequence; ev (if given) holds an event slot before every pass
// and after the last, recorded as marker packets where the slot exists.  For
// the pass at position `bind`, if it launches the pipelined kernel, slots
// bind and bind + 1 are instead bound to that launch's own start and end.
pafc_status run_sequence(pafc_plan_t p, const std::vector<Pass>& seq, const void* x, void* y,
                         hipStream_t s, hipEvent_t* ev = nullptr, int bind = -1) {
  const PlanCore& P = p->P;
  const bool dbl = P.dtype == PAFC_C128;
  const void* cur = x;
  size_t k = 0;
  const bool bound = ev && bind >= 0 && bind < (int)seq.size() && pass_binds_events(seq[bind]);
  if (!(bound && bind == 0)) PAFC_TRY(rec(ev, 0, s));
  for (const Pass& ps : seq) {
    if (bound && (int)k == bind) {
      PAFC_TRY(run_pass(p, ps, cur, y, s, ev[k], ev[k + 1]));
      cur = y;
      ++k;
      continue;
    }
    if (ps.kind == 0) {
      PAFC_TRY(run_pass(p, ps, cur, y, s));
      cur = y;
    } else if (ps.kind == 1) {
      PAFC_TRY(from_hip(launch_mul(dbl, cur, p->d_H, y, P.N, 1.0 / (double)P.N, p->nt_h, s)));
      cur = y;
    } else if (ps.kind == 2) {
      if (ps.perm_dir == 1) {
        PAFC_TRY(run_permute(p, 1, cur, p->d_scratch, p->d_H, s));
        cur = p->d_scratch;
      } else {
        PAFC_TRY(run_permute(p, 2, cur, y, nullptr, s));
        cur = y;
      }
    }
    ++k;
    PAFC_TRY(rec(ev, k, s));
  }
  if (cur != y) return PAFC_ERROR_DEVICE;
  return PAFC_SUCCESS;
}

int64_t pass_bytes(const PlanCore& P, const Pass& ps) {
  const int64_t ne = P.N * (int64_t)P.elem;
  if (ps.kind == 0) return 2 * ne + (ps.mid ? ne : 0);
  if (ps.kind == 1) return 3 * ne;
  if (ps.kind == 2) return 2 * ne + (ps.perm_dir == 1 ? ne : 0);
  return 0;
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// Prime-factor route (Sec. "Prime factor framework").  For n with pairwise
// coprime factors N_q, j -> (j mod N_q)_q is a ring isomorphism Z_n ->
// prod Z_{N_q} (Chinese remainder theorem), so (j - k) mod n maps to the
// componentwise differences and the length-n circular convolution is the
// grid convolution of the reindexed arrays.

// The powers of 2, 3 and 5 in n, ascending; false unless n is {2,3,5}-smooth
// with at least two of them.
bool pfa_factors(int64_t n, std::vector<int64_t>* f) {
  f->clear();
  for (int p : {2, 3, 5}) {
    int64_t q = 1;
    while (n % p == 0) {
      n /= p;
      q *= p;
    }
    if (q > 1) f->push_back(q);
  }
  std::sort(f->begin(), f->end());
  return n == 1 && f->size() >= 2;
}

// a^-1 mod m for coprime a, m (m >= 1)
int64_t inv_mod(int64_t a, int64_t m) {
  int64_t g = m, x = 0, g1 = a % m, x1 = 1;
  while (g1 != 0) {
    const int64_t q = g / g1;
    int64_t t = g - q * g1;
    g = g1;
    g1 = t;
    t = x - q * x1;
    x = x1;
    x1 = t;
  }
  x %= m;
  return x < 0 ? x + m : x;
}

// which 0: the CRT input map (x -> grid); 1: the output map of the spectrum
pafc_status pfa_gather(pafc_plan_t p, const void* in, void* out, int which, hipStream_t s) {
  const uint32_t* N = p->pfa_N;
  if (which == 0)
    return from_hip(launch_pfa_map(p->P.dtype == PAFC_C128, 0, in, out, N[0], N[1], N[2],
                                   p->pfa_uinv, s));
  const uint32_t* t = p->d_pfa_tab + (size_t)which * (N[0] + N[1] + N[2]);
  return from_hip(launch_pfa_gather(p->P.dtype == PAFC_C128, in, out, t, t + N[0], t + N[0] + N[1],
                                    N[1], N[2], (uint32_t)p->P.N, s));
}

pafc_status pfa_scatter(pafc_plan_t p, const void* in, void* out, hipStream_t s) {
  const uint32_t* N = p->pfa_N;
  return from_hip(launch_pfa_map(p->P.dtype == PAFC_C128, 1, in, out, N[0], N[1], N[2],
                                 p->pfa_uinv, s));
}

// gather, the grid convolution in place, scatter; events (when given) before
// the gather and after every launch
pafc_status pfa_convolve(pafc_plan_t p, const void* x, void* y, hipStream_t s,
                         hipEvent_t* ev = nullptr) {
  PAFC_TRY(rec(ev, 0, s));
  PAFC_TRY(pfa_gather(p, x, p->d_scratch, 0, s));
  PAFC_TRY(run_sequence(p->inner, p->inner->P.conv, p->d_scratch, p->d_scratch, s,
                        ev ? ev + 1 : nullptr));
  PAFC_TRY(pfa_scatter(p, p->d_scratch, y, s));
  PAFC_TRY(rec(ev, p->inner->P.conv.size() + 2, s));
  return PAFC_SUCCESS;
}

pafc_status plan_prime_factor(pafc_plan_t* out, int ndim, const int64_t* dims, const int* radix,
                              pafc_dtype dtype, pafc_variant variant, void* hip_stream) {
  if (ndim != 1 || !dims || (radix && radix[0] != 0)) return PAFC_ERROR_INVALID_VALUE;
  if (dtype != PAFC_C64 && dtype != PAFC_C128) return PAFC_ERROR_INVALID_VALUE;
  const int64_t n = dims[0];
  if (n < 2) return PAFC_ERROR_INVALID_VALUE;
  std::vector<int64_t> f;
  if (n >= ((int64_t)1 << 31) || !pfa_factors(n, &f)) return PAFC_ERROR_UNSUPPORTED_SIZE;
  pafc_plan_t p = new (std::nothrow) pafc_plan_s;
  if (!p) return PAFC_ERROR_OUT_OF_MEMORY;
  p->P.ndim = 1;
  p->P.dims[0] = n;
  p->P.N = n;
  p->P.dtype = dtype;
  p->P.variant = variant;
  p->P.elem = dtype == PAFC_C128 ? 16 : 8;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return PAFC_ERROR_DEVICE;
  }
  pafc_status st = pafc_plan(&p->inner, (int)f.size(), f.data(), nullptr, dtype,
                             variant == PAFC_PRIME_FACTOR ? PAFC_PERM_FREE : PAFC_EXPLICIT_PERM,
                             hip_stream);
  if (st != PAFC_SUCCESS) {
    p->inner = nullptr;
    free_plan(p);
    return st;
  }
  const size_t nf = f.size();
  for (size_t q = 0; q < nf; ++q) p->pfa_N[3 - nf + q] = (uint32_t)f[q];
  p->pfa_uinv = (uint32_t)inv_mod((int64_t)p->pfa_N[0] * p->pfa_N[1] % p->pfa_N[2], p->pfa_N[2]);
  // tables: t_q[j] = j c_q mod n, c_q = e_q (CRT basis: 1 mod N_q, 0 mod the
  // others) for the input map, c_q = n / N_q for the spectrum's output map
  const uint32_t tot = p->pfa_N[0] + p->pfa_N[1] + p->pfa_N[2];
  std::vector<uint32_t> tab((size_t)2 * tot);
  for (int which = 0; which < 2; ++which) {
    size_t at = (size_t)which * tot;
    for (int q = 0; q < 3; ++q) {
      const int64_t Nq = p->pfa_N[q];
      const int64_t m = n / Nq;
      const int64_t c = Nq == 1 ? 0 : which == 0 ? (m % n) * inv_mod(m % Nq, Nq) % n : m;
      for (int64_t j = 0; j < Nq; ++j) tab[at++] = (uint32_t)((j * c) % n);
    }
  }
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = hipMalloc((void**)&p->d_pfa_tab, tab.size() * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&p->d_scratch, (size_t)n * p->P.elem);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->d_pfa_tab, tab.data(), tab.size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host table dies here
  if (e != hipSuccess) {
    free_plan(p);
    return from_hip(e);
  }
  p->bytes = p->inner->bytes + tab.size() * sizeof(uint32_t) + (size_t)n * p->P.elem;
  *out = p;
  return PAFC_SUCCESS;
}

// ---------------------------------------------------------------------------
// Bluestein route (Sec. "Rader's and Bluestein's frameworks") for a 1-D
// length with a prime factor above 5: the length-n DFT as a length-m
// circular convolution, m the smallest {2,3,5}-smooth length >= 2n - 1,
// which runs on a permutation-avoiding inner plan (or the comparison
// variants).  A convolution: chirp-in, inner convolution, chirp product with
// the spectrum, inner convolution (the inverse DFT through conjugation),
// chirp-out.

bool smooth235(int64_t n) {
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

int64_t smooth_at_least(int64_t v) {
  for (int64_t m = v;; ++m)
    if (smooth235(m)) return m;
}

bool is_prime(int64_t n) {
  if (n < 2) return false;
  for (int64_t d = 2; d * d <= n; ++d)
    if (n % d == 0) return false;
  return true;
}

bool is_rader_case(int ndim, const int64_t* dims, const int* radix, int variant) {
  return ndim == 1 && dims && dims[0] >= 7 && dims[0] <= ((int64_t)1 << 30) &&
         (!radix || radix[0] == 0) && variant >= PAFC_PERM_FREE &&
         variant <= PAFC_PERM_FREE_UNFUSED && !smooth235(dims[0]) && smooth235(dims[0] - 1) &&
         is_prime(dims[0]) && env_int("PAFC_BLUESTEIN", 0) == 0;
}

bool is_bluestein_case(int ndim, const int64_t* dims, const int* radix, int variant) {
  return ndim == 1 && dims && dims[0] >= 2 && !smooth235(dims[0]) && (!radix || radix[0] == 0) &&
         variant >= PAFC_PERM_FREE && variant <= PAFC_PERM_FREE_UNFUSED &&
         !is_rader_case(ndim, dims, radix, variant);
}

bool is_bluestein(pafc_plan_t p) { return p->blue_m > 0; }
bool is_rader(pafc_plan_t p) { return p->rader_g > 0; }
bool is_prime_factor(pafc_plan_t p) { return p->inner && p->blue_m == 0 && p->rader_g == 0; }

pafc_status blue_stage(pafc_plan_t p, int stage, const void* src, void* dst, hipStream_t s) {
  return from_hip(launch_bluestein(p->P.dtype == PAFC_C128, stage, src, p->d_chirp, dst, p->d_hn,
                                   p->P.N, p->blue_m, 1.0 / (double)p->P.N, s));
}

// events (when given) before the first launch and after every launch
pafc_status blue_convolve(pafc_plan_t p, const void* x, void* y, hipStream_t s,
                          hipEvent_t* ev = nullptr) {
  const size_t k = p->inner->P.conv.size();
  void* b = p->d_scratch;
  PAFC_TRY(rec(ev, 0, s));
  PAFC_TRY(blue_stage(p, 0, x, b, s));
  PAFC_TRY(run_sequence(p->inner, p->inner->P.conv, b, b, s, ev ? ev + 1 : nullptr));
  PAFC_TRY(blue_stage(p, 2, b, b, s));
  PAFC_TRY(rec(ev, k + 2, s));
  PAFC_TRY(run_sequence(p->inner, p->inner->P.conv, b, b, s, ev ? ev + k + 2 : nullptr));
  PAFC_TRY(blue_stage(p, 3, b, y, s));
  PAFC_TRY(rec(ev, 2 * k + 3, s));
  return PAFC_SUCCESS;
}

// the filter's natural-order spectrum by the forward Bluestein DFT
pafc_status blue_set_filter(pafc_plan_t p, const void* h, pafc_filter_domain domain,
                            hipStream_t s) {
  if (domain == PAFC_FILTER_SPECTRAL_NATURAL)
    return from_hip(hipMemcpyAsync(p->d_hn, h, (size_t)p->P.N * p->P.elem,
                                   hipMemcpyDeviceToDevice, s));
  void* b = p->d_scratch;
  PAFC_TRY(blue_stage(p, 0, h, b, s));
  PAFC_TRY(run_sequence(p->inner, p->inner->P.conv, b, b, s));
  return blue_stage(p, 1, b, p->d_hn, s);
}

pafc_status plan_bluestein(pafc_plan_t* out, int64_t n, pafc_dtype dtype, pafc_variant variant,
                           void* hip_stream) {
  if (dtype != PAFC_C64 && dtype != PAFC_C128) return PAFC_ERROR_INVALID_VALUE;
  if (n > ((int64_t)1 << 29)) return PAFC_ERROR_UNSUPPORTED_SIZE;
  const int64_t m = smooth_at_least(2 * n - 1);
  pafc_plan_t p = new (std::nothrow) pafc_plan_s;
  if (!p) return PAFC_ERROR_OUT_OF_MEMORY;
  p->P.ndim = 1;
  p->P.dims[0] = n;
  p->P.N = n;
  p->P.dtype = dtype;
  p->P.variant = variant;
  p->P.elem = dtype == PAFC_C128 ? 16 : 8;
  p->blue_m = m;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return PAFC_ERROR_DEVICE;
  }
  pafc_status st = pafc_plan(&p->inner, 1, &m, nullptr, dtype, variant, hip_stream);
  if (st != PAFC_SUCCESS) {
    p->inner = nullptr;
    free_plan(p);
    return st;
  }
  // chirp c_j = w_{2n}^{j^2 mod 2n} (FP64 with exact octant reduction, FP32
  // plans round it once) and the inner filter g: conj(c_d) at offsets d and
  // m - d for 0 <= d < n, zero elsewhere
  std::vector<double> c64((size_t)n * 2), g64((size_t)m * 2, 0.0);
  for (int64_t j = 0; j < n; ++j) {
    const int64_t e = (int64_t)(((unsigned __int128)j * (unsigned __int128)j) % (unsigned __int128)(2 * n));
    omega64(2 * n, e, &c64[(size_t)j * 2], &c64[(size_t)j * 2 + 1]);
    g64[(size_t)j * 2] = c64[(size_t)j * 2];
    g64[(size_t)j * 2 + 1] = -c64[(size_t)j * 2 + 1];
    if (j > 0) {
      g64[(size_t)(m - j) * 2] = c64[(size_t)j * 2];
      g64[(size_t)(m - j) * 2 + 1] = -c64[(size_t)j * 2 + 1];
    }
  }
  std::vector<float> c32, g32;
  const void* ch = c64.data();
  const void* gh = g64.data();
  if (dtype == PAFC_C64) {
    c32.assign(c64.begin(), c64.end());
    g32.assign(g64.begin(), g64.end());
    ch = c32.data();
    gh = g32.data();
  }
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t eb = p->P.elem;
  hipError_t e = hipMalloc(&p->d_chirp, (size_t)n * eb);
  if (e == hipSuccess) e = hipMalloc(&p->d_hn, (size_t)n * eb);
  if (e == hipSuccess) e = hipMalloc(&p->d_scratch, (size_t)m * eb);
  if (e == hipSuccess) e = hipMemcpyAsync(p->d_chirp, ch, (size_t)n * eb, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(p->d_scratch, gh, (size_t)m * eb, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    free_plan(p);
    return from_hip(e);
  }
  st = pafc_set_filter(p->inner, p->d_scratch, PAFC_FILTER_SPATIAL, hip_stream);
  if (st == PAFC_SUCCESS) st = from_hip(hipStreamSynchronize(s));  // host tables die here
  if (st != PAFC_SUCCESS) {
    free_plan(p);
    return st;
  }
  p->bytes = p->inner->bytes + (2 * (size_t)n + (size_t)m) * eb;
  *out = p;
  return PAFC_SUCCESS;
}

std::string describe_bluestein(int64_t n, pafc_dtype dtype, pafc_variant variant,
                               pafc_status* st) {
  *st = PAFC_SUCCESS;
  if (dtype != PAFC_C64 && dtype != PAFC_C128) {
    *st = PAFC_ERROR_INVALID_VALUE;
    return "";
  }
  if (n > ((int64_t)1 << 29)) {
    *st = PAFC_ERROR_UNSUPPORTED_SIZE;
    return "";
  }
  const int64_t m = smooth_at_least(2 * n - 1);
  PlanCore G;
  *st = plan_core(G, 1, &m, nullptr, dtype, variant);
  if (*st != PAFC_SUCCESS) return "";
  const int64_t eb = dtype == PAFC_C128 ? 16 : 8;
  char b[256];
  std::string s = "{";
  snprintf(b, sizeof(b), "\"ndim\": 1, \"dims\": [%lld], \"dtype\": \"%s\", \"variant\": %d, "
           "\"bluestein_m\": %lld, \"conv_passes\": [\"bluestein chirp-in\"",
           (long long)n, dtype == PAFC_C128 ? "c128" : "c64", (int)variant, (long long)m);
  s += b;
  for (auto& ps : G.conv) s += ", \"" + ps.label + "\"";
  s += ", \"bluestein chirp product\"";
  for (auto& ps : G.conv) s += ", \"" + ps.label + "\"";
  snprintf(b, sizeof(b), ", \"bluestein chirp-out\"], \"hbm_bytes_conv\": %lld, "
           "\"hbm_bytes_forward\": %lld, \"N\": %lld, \"inner\": ",
           (long long)(2 * G.hbm_conv + ((2 * n + m) + (2 * m + 2 * n) + (m + 2 * n)) * eb), (long long)(G.hbm_conv + (2 * n + m) * eb + 2 * n * eb),
           (long long)n);
  s += b;
  s += describe_core(G) + "}";
  return s;
}

// ---------------------------------------------------------------------------
// Rader route (Sec. "Rader's and Bluestein's frameworks") for a prime length
// p whose p - 1 is {2,3,5}-smooth: the DFT at the nonzero frequencies is a
// length p - 1 circular convolution after reindexing by powers of a
// generator g; that convolution runs on a permutation-avoiding inner plan.
// The spectrum stays in generator order between the two inner convolutions,
// so one evaluation permutes twice (gather in, scatter out) where undoing
// each reindexing would take four.  A convolution: gather, inner
// convolution, product with the spectrum (+ block sums), the two DC
// constants, inner convolution (the inverse DFT through conjugation),
// scatter.

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) {
  return (uint64_t)((unsigned __int128)a * b % m);
}

uint64_t powmod(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  for (b %= m; e; e >>= 1, b = mulmod(b, b, m))
    if (e & 1) r = mulmod(r, b, m);
  return r;
}

// smallest generator of the multiplicative group mod the prime p (p - 1
// has prime factors in {2, 3, 5} only)
int64_t primitive_root(int64_t p) {
  for (int64_t g = 2; g < p; ++g) {
    bool ok = true;
    for (int q : {2, 3, 5})
      if ((p - 1) % q == 0 && powmod((uint64_t)g, (uint64_t)((p - 1) / q), (uint64_t)p) == 1)
        ok = false;
    if (ok) return g;
  }
  return 0;
}

pafc_status rader_stage(pafc_plan_t p, int stage, int mode, const void* src, const void* x,
                        void* dst, hipStream_t s) {
  const uint32_t n = (uint32_t)p->P.N;
  const double* acc = p->d_rader_acc;
  return from_hip(launch_rader(p->P.dtype == PAFC_C128, stage, mode, src, x, dst, p->d_hn,
                               p->d_rader_tab, p->d_rader_tab + (n - 1), p->d_rader_acc,
                               (void*)(acc + 4 * (size_t)kRaderBlocks), n, 1.0 / (double)n, s));
}

// events (when given) before the first launch and after every launch
pafc_status rader_convolve(pafc_plan_t p, const void* x, void* y, hipStream_t s,
                           hipEvent_t* ev = nullptr) {
  const size_t k = p->inner->P.conv.size();
  void* b = p->d_scratch;
  PAFC_TRY(rec(ev, 0, s));
  PAFC_TRY(rader_stage(p, 0, 0, x, nullptr, b, s));
  PAFC_TRY(run_sequence(p->inner, p->inner->P.conv, b, b, s, ev ? ev + 1 : nullptr));
  PAFC_TRY(rader_stage(p, 1, 1, nullptr, x, b, s));
  PAFC_TRY(rec(ev, k + 2, s));
  PAFC_TRY(rader_stage(p, 2, 1, nullptr, x, nullptr, s));
  PAFC_TRY(rec(ev, k + 3, s));
  PAFC_TRY(run_sequence(p->inner, p->inner->P.conv, b, b, s, ev ? ev + k + 3 : nullptr));
  PAFC_TRY(rader_stage(p, 3, 0, b, nullptr, y, s));
  PAFC_TRY(rec(ev, 2 * k + 4, s));
  return PAFC_SUCCESS;
}

// the filter's spectrum in generator order: by the forward Rader DFT, or
// reordered from a natural-order spectrum
pafc_status rader_set_filter(pafc_plan_t p, const void* h, pafc_filter_domain domain,
                             hipStream_t s) {
  if (domain == PAFC_FILTER_SPECTRAL_NATURAL) return rader_stage(p, 4, 0, h, nullptr, nullptr, s);
  void* b = p->d_scratch;
  PAFC_TRY(rader_stage(p, 0, 0, h, nullptr, b, s));
  PAFC_TRY(run_sequence(p->inner, p->inner->P.conv, b, b, s));
  PAFC_TRY(rader_stage(p, 1, 0, nullptr, h, b, s));
  return rader_stage(p, 2, 0, nullptr, h, nullptr, s);
}

pafc_status plan_rader(pafc_plan_t* out, int64_t n, pafc_dtype dtype, pafc_variant variant,
                       void* hip_stream) {
  if (dtype != PAFC_C64 && dtype != PAFC_C128) return PAFC_ERROR_INVALID_VALUE;
  const int64_t P1 = n - 1;
  const int64_t g = primitive_root(n);
  if (g == 0) return PAFC_ERROR_UNSUPPORTED_SIZE;
  pafc_plan_t p = new (std::nothrow) pafc_plan_s;
  if (!p) return PAFC_ERROR_OUT_OF_MEMORY;
  p->P.ndim = 1;
  p->P.dims[0] = n;
  p->P.N = n;
  p->P.dtype = dtype;
  p->P.variant = variant;
  p->P.elem = dtype == PAFC_C128 ? 16 : 8;
  p->rader_g = g;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return PAFC_ERROR_DEVICE;
  }
  pafc_status st = pafc_plan(&p->inner, 1, &P1, nullptr, dtype, variant, hip_stream);
  if (st != PAFC_SUCCESS) {
    p->inner = nullptr;
    free_plan(p);
    return st;
  }
  // tables and the inner filter b_l = w_n^{g^{-l}} (FP64 with exact octant
  // reduction; FP32 plans round it once)
  std::vector<uint32_t> tab((size_t)(P1 + n), 0);
  uint64_t gm = 1;
  for (int64_t m = 0; m < P1; ++m, gm = mulmod(gm, (uint64_t)g, (uint64_t)n)) {
    tab[(size_t)m] = (uint32_t)gm;
    tab[(size_t)(P1 + (int64_t)gm)] = (uint32_t)((P1 - m) % P1);
  }
  std::vector<double> b64((size_t)P1 * 2);
  for (int64_t l = 0; l < P1; ++l) {
    const int64_t e = tab[(size_t)((P1 - l) % P1)];
    omega64(n, e, &b64[(size_t)l * 2], &b64[(size_t)l * 2 + 1]);
  }
  std::vector<float> b32;
  const void* bh = b64.data();
  if (dtype == PAFC_C64) {
    b32.assign(b64.begin(), b64.end());
    bh = b32.data();
  }
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t eb = p->P.elem;
  hipError_t e = hipMalloc(&p->d_hn, (size_t)n * eb);
  if (e == hipSuccess) e = hipMalloc(&p->d_scratch, (size_t)P1 * eb);
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_rader_tab, tab.size() * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_rader_acc, (4 * (size_t)kRaderBlocks + 8) * sizeof(double));
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->d_rader_tab, tab.data(), tab.size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(p->d_scratch, bh, (size_t)P1 * eb, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    free_plan(p);
    return from_hip(e);
  }
  st = pafc_set_filter(p->inner, p->d_scratch, PAFC_FILTER_SPATIAL, hip_stream);
  if (st == PAFC_SUCCESS) st = from_hip(hipStreamSynchronize(s));  // host tables die here
  if (st != PAFC_SUCCESS) {
    free_plan(p);
    return st;
  }
  p->bytes = p->inner->bytes + ((size_t)n + (size_t)P1) * eb +
             tab.size() * sizeof(uint32_t) + (4 * (size_t)kRaderBlocks + 8) * sizeof(double);
  *out = p;
  return PAFC_SUCCESS;
}

// algorithmic bytes of the Rader stages: gather (x, table, a), product
// (u, spectrum, w), constants (block sums), scatter (v, table, y)
void rader_stage_bytes(int64_t n, int64_t eb, int64_t* gather, int64_t* product,
                       int64_t* fin, int64_t* scatter) {
  const int64_t P1 = n - 1;
  *gather = (2 * eb + 4) * P1;
  *product = 3 * eb * P1;
  *fin = 4 * 8 * ((P1 / 2 + 1 + 255) / 256 < (int64_t)kRaderBlocks ? (P1 / 2 + 1 + 255) / 256
                                                                    : (int64_t)kRaderBlocks);
  *scatter = (2 * eb + 4) * n;
}

std::string describe_rader(int64_t n, pafc_dtype dtype, pafc_variant variant, pafc_status* st) {
  *st = PAFC_SUCCESS;
  if (dtype != PAFC_C64 && dtype != PAFC_C128) {
    *st = PAFC_ERROR_INVALID_VALUE;
    return "";
  }
  const int64_t P1 = n - 1;
  PlanCore G;
  *st = plan_core(G, 1, &P1, nullptr, dtype, variant);
  if (*st != PAFC_SUCCESS) return "";
  const int64_t eb = dtype == PAFC_C128 ? 16 : 8;
  int64_t bg, bp, bf, bs;
  rader_stage_bytes(n, eb, &bg, &bp, &bf, &bs);
  char b[320];
  std::string s = "{";
  snprintf(b, sizeof(b), "\"ndim\": 1, \"dims\": [%lld], \"dtype\": \"%s\", \"variant\": %d, "
           "\"rader_generator\": %lld, \"rader_inner\": %lld, \"conv_passes\": [\"rader gather\"",
           (long long)n, dtype == PAFC_C128 ? "c128" : "c64", (int)variant,
           (long long)primitive_root(n), (long long)P1);
  s += b;
  for (auto& ps : G.conv) s += ", \"" + ps.label + "\"";
  s += ", \"rader product\", \"rader constants\"";
  for (auto& ps : G.conv) s += ", \"" + ps.label + "\"";
  // filter per call: gather, inner convolution, spectrum (u in, spectrum out)
  snprintf(b, sizeof(b), ", \"rader scatter\"], \"hbm_bytes_conv\": %lld, "
           "\"hbm_bytes_forward\": %lld, \"N\": %lld, \"inner\": ",
           (long long)(2 * G.hbm_conv + bg + bp + bf + bs),
           (long long)(G.hbm_conv + bg + 2 * eb * P1 + bf), (long long)n);
  s += b;
  s += describe_core(G) + "}";
  return s;
}

// ------------------------------------------------------------ profiling

// launches of one convolution, in the order the profiling calls report them
int route_launches(pafc_plan_t p) {
  if (is_bluestein(p)) return 2 * (int)p->inner->P.conv.size() + 3;
  if (is_rader(p)) return 2 * (int)p->inner->P.conv.size() + 4;
  if (p->inner) return (int)p->inner->P.conv.size() + 2;
  return (int)p->P.conv.size();
}

pafc_status route_convolve(pafc_plan_t p, const void* x, void* y, hipStream_t s,
                           hipEvent_t* ev, int bind) {
  if (is_bluestein(p)) return blue_convolve(p, x, y, s, ev);
  if (is_rader(p)) return rader_convolve(p, x, y, s, ev);
  if (p->inner) return pfa_convolve(p, x, y, s, ev);
  return run_sequence(p, p->P.conv, x, y, s, ev, bind);
}

// algorithmic HBM bytes of launch i of one convolution
int64_t route_pass_bytes(pafc_plan_t p, int i) {
  const int64_t eb = p->P.elem, N = p->P.N;
  if (is_bluestein(p)) {
    const auto& seq = p->inner->P.conv;
    const int k = (int)seq.size(), n = 2 * k + 3;
    const int64_t m = p->blue_m;
    if (i == 0) return (2 * N + m) * eb;              // chirp-in
    if (i == k + 1) return (2 * m + 2 * N) * eb;      // chirp product
    if (i == n - 1) return (m + 2 * N) * eb;          // chirp-out
    return pass_bytes(p->inner->P, seq[(size_t)((i - 1) % (k + 1))]);
  }
  if (is_rader(p)) {
    const auto& seq = p->inner->P.conv;
    const int k = (int)seq.size(), n = 2 * k + 4;
    int64_t bg, bp, bf, bs;
    rader_stage_bytes(N, eb, &bg, &bp, &bf, &bs);
    if (i == 0) return bg;
    if (i == k + 1) return bp;
    if (i == k + 2) return bf;
    if (i == n - 1) return bs;
    return pass_bytes(p->inner->P, seq[(size_t)(i <= k ? i - 1 : i - k - 3)]);
  }
  if (p->inner) {  // prime-factor: gather, grid passes, scatter
    const int n = (int)p->inner->P.conv.size() + 2;
    if (i == 0 || i == n - 1) return 2 * N * eb;
    return pass_bytes(p->inner->P, p->inner->P.conv[(size_t)i - 1]);
  }
  return pass_bytes(p->P, p->P.conv[(size_t)i]);
}

// `reps` convolutions with timing events at launch boundaries.  sel < 0:
// an event before every launch and after the last, and ms_per_pass[k] the
// mean of launch k.  sel >= 0: events at the start of every repetition and
// around launch sel only (fewer event packets in the stream), *ms_sel its
// mean.  ms_per_rep[r] (may be NULL): start of repetition r to the start of
// the next (to the end of the last).
pafc_status profile_impl(pafc_plan_t p, const void* x, void* y, hipStream_t s, int reps, int sel,
                         double* ms_per_pass, double* ms_per_rep, double* ms_sel) {
  const int n = route_launches(p);
  const size_t stride = (size_t)n + 1;
  std::vector<hipEvent_t> ev(stride * (size_t)reps, nullptr);
  // one launch timed: events around it, and at the start of every
  // repetition (and the end of the last) only when per-repetition times are
  // asked for; a pipelined launch carries its pair itself
  // A plan of one launch, timed without per-repetition times, takes one
  // pair over the whole sequence instead (start of the first launch, end of
  // the last) and reports its span over reps: the gaps between launches
  // count as launch time, and no launch but the first and the last carries
  // an event.
  const bool span = sel == 0 && n == 1 && !ms_per_rep && reps > 1;
  auto want = [&](int r, int k) {
    if (span) return (r == 0 && k == 0) || (r == reps - 1 && k == 1);
    return sel < 0 || k == sel || k == sel + 1 ||
           (ms_per_rep && (k == 0 || (k == n && r == reps - 1)));
  };
  pafc_status st = PAFC_SUCCESS;
  for (int r = 0; r < reps; ++r)
    for (int k = 0; k <= n && st == PAFC_SUCCESS; ++k)
      if (want(r, k)) st = from_hip(timing_event(&ev[(size_t)r * stride + (size_t)k]));
  for (int r = 0; r < reps && st == PAFC_SUCCESS; ++r)
    st = route_convolve(p, x, y, s, ev.data() + (size_t)r * stride, sel);
  if (st == PAFC_SUCCESS) st = from_hip(hipStreamSynchronize(s));
  auto elapsed = [&](hipEvent_t a, hipEvent_t b, double* out) {
    float ms = 0;
    if (st == PAFC_SUCCESS) st = from_hip(hipEventElapsedTime(&ms, a, b));
    *out = ms;
  };
  if (span) {
    double ms = 0;
    elapsed(ev[0], ev[(size_t)(reps - 1) * stride + 1], &ms);
    *ms_sel = ms / reps;
  }
  for (int k = 0; k < n && st == PAFC_SUCCESS && !span; ++k) {
    if (sel >= 0 && k != sel) continue;
    double tot = 0, ms = 0;
    for (int r = 0; r < reps; ++r) {
      elapsed(ev[(size_t)r * stride + (size_t)k], ev[(size_t)r * stride + (size_t)k + 1], &ms);
      tot += ms;
    }
    if (sel < 0) ms_per_pass[k] = tot / reps;
    else *ms_sel = tot / reps;
  }
  for (int r = 0; r < reps && ms_per_rep; ++r) {
    hipEvent_t end = ev[(size_t)r * stride + (size_t)n];
    if (!end) end = ev[(size_t)(r + 1) * stride];
    elapsed(ev[(size_t)r * stride], end, &ms_per_rep[r]);
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  return st;
}

std::string describe_prime_factor(int64_t n, pafc_dtype dtype, pafc_variant variant,
                                  pafc_status* st) {
  std::vector<int64_t> f;
  *st = PAFC_SUCCESS;
  if (n < 2) {
    *st = PAFC_ERROR_INVALID_VALUE;
    return "";
  }
  if (n >= ((int64_t)1 << 31) || !pfa_factors(n, &f)) {
    *st = PAFC_ERROR_UNSUPPORTED_SIZE;
    return "";
  }
  PlanCore G;
  *st = plan_core(G, (int)f.size(), f.data(), nullptr, dtype,
                  variant == PAFC_PRIME_FACTOR ? PAFC_PERM_FREE : PAFC_EXPLICIT_PERM);
  if (*st != PAFC_SUCCESS) return "";
  const int64_t elem = dtype == PAFC_C128 ? 16 : 8;
  char b[256];
  std::string s = "{";
  snprintf(b, sizeof(b), "\"ndim\": 1, \"dims\": [%lld], \"dtype\": \"%s\", \"variant\": %d, "
           "\"prime_factor_grid\": [", (long long)n, dtype == PAFC_C128 ? "c128" : "c64", (int)variant);
  s += b;
  for (size_t q = 0; q < f.size(); ++q) {
    snprintf(b, sizeof(b), "%s%lld", q ? ", " : "", (long long)f[q]);
    s += b;
  }
  s += "], \"conv_passes\": [\"pfa gather (CRT input map)\"";
  for (auto& ps : G.conv) s += ", \"" + ps.label + "\"";
  snprintf(b, sizeof(b), ", \"pfa scatter\"], \"hbm_bytes_conv\": %lld, \"hbm_bytes_forward\": %lld, "
           "\"N\": %lld, \"grid\": ",
           (long long)(G.hbm_conv + 4 * n * elem), (long long)(G.hbm_fwd + 2 * n * elem), (long long)n);
  s += b;
  s += describe_core(G) + "}";
  return s;
}

// A spectrum produced in plan layout (natural-order input, symbols) for a
// plan that stores it tile-major: `produce` writes the plan layout into the
// plan's staging array, which is then reordered into the spectrum (the two
// layouts place a tile's values differently, so it cannot be done in place).
template <typename F>
pafc_status via_plan_layout(pafc_plan_t p, hipStream_t s, F produce) {
  const PlanCore& P = p->P;
  const Pass& m = P.conv[(size_t)p->mid_pass];
  PAFC_TRY(produce(p->d_scratch));
  return from_hip(launch_pipe_htm(P.dtype == PAFC_C128, m.pipe_r, m.pipe_g, m.pipe_ng,
                                  (int)m.a.mode, p->d_descs + m.desc, m.a.ntiles, m.pipe_threads,
                                  p->d_scratch, p->d_H, s));
}

// The filter's forward transform for a plan that stores the spectrum
// tile-major: all forward passes but the last in the staging array, the
// last one from there into the spectrum in tile-major order.
pafc_status forward_tile_major(pafc_plan_t p, const void* h, hipStream_t s) {
  const std::vector<Pass> head(p->fwd_tm.begin(), p->fwd_tm.end() - 1);
  const void* src = h;
  if (!head.empty()) {
    PAFC_TRY(run_sequence(p, head, h, p->d_scratch, s));
    src = p->d_scratch;
  }
  return run_pass(p, p->fwd_tm.back(), src, p->d_H, s);
}

}  // namespace

extern "C" {

const char* pafc_status_string(pafc_status s) {
  switch (s) {
    case PAFC_SUCCESS: return "success";
    case PAFC_ERROR_INVALID_VALUE: return "invalid value";
    case PAFC_ERROR_UNSUPPORTED_SIZE: return "unsupported size";
    case PAFC_ERROR_OUT_OF_MEMORY: return "out of device memory";
    case PAFC_ERROR_DEVICE: return "device error";
    case PAFC_ERROR_FILTER_NOT_SET: return "filter not set";
  }
  return "unknown status";
}

pafc_status pafc_describe(int ndim, const int64_t* dims, const int* radix, pafc_dtype dtype,
                          pafc_variant variant, char* buf, size_t cap, size_t* needed) {
  std::string s;
  if (is_rader_case(ndim, dims, radix, variant)) {
    pafc_status st;
    s = describe_rader(dims[0], dtype, variant, &st);
    PAFC_TRY(st);
  } else if (is_bluestein_case(ndim, dims, radix, variant)) {
    pafc_status st;
    s = describe_bluestein(dims[0], dtype, variant, &st);
    PAFC_TRY(st);
  } else if (variant == PAFC_PRIME_FACTOR || variant == PAFC_PRIME_FACTOR_EXPLICIT) {
    if (ndim != 1 || !dims || (radix && radix[0] != 0)) return PAFC_ERROR_INVALID_VALUE;
    if (dtype != PAFC_C64 && dtype != PAFC_C128) return PAFC_ERROR_INVALID_VALUE;
    pafc_status st;
    s = describe_prime_factor(dims[0], dtype, variant, &st);
    PAFC_TRY(st);
  } else {
    PlanCore P;
    PAFC_TRY(plan_core(P, ndim, dims, radix, dtype, variant));
    s = describe_core(P);
  }
  if (needed) *needed = s.size() + 1;
  if (buf && cap > 0) {
    size_t n = std::min(cap - 1, s.size());
    memcpy(buf, s.data(), n);
    buf[n] = 0;
  }
  return PAFC_SUCCESS;
}

}  // extern "C"

namespace {

// A plan of a {2,3,5}-smooth shape under the given limits (pafc_plan's
// direct route).
pafc_status make_plan(pafc_plan_t* out, int ndim, const int64_t* dims, const int* radix,
                      pafc_dtype dtype, pafc_variant variant, void* hip_stream,
                      const PlanLimits& lim) {
  *out = nullptr;
  pafc_plan_t p = new (std::nothrow) pafc_plan_s;
  if (!p) return PAFC_ERROR_OUT_OF_MEMORY;
  pafc_status st = plan_core(p->P, ndim, dims, radix, dtype, variant, lim);
  if (st != PAFC_SUCCESS) {
    delete p;
    return st;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  const PlanCore& P = p->P;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return PAFC_ERROR_DEVICE;
  }
  // twiddle tables (FP64 on the host; FP32 plans take the rounded values)
  std::vector<double> tw64((size_t)P.tw_elems * 2);
  for (auto& kv : P.tw) {
    const TwTable& t = kv.second;
    if (t.hi_off < 0) {
      for (int64_t e = 0; e < t.n; ++e)
        omega64(t.n, e, &tw64[(size_t)(t.lo_off + e) * 2], &tw64[(size_t)(t.lo_off + e) * 2 + 1]);
    } else {
      const int64_t nlo = (int64_t)1 << t.bits;
      const int64_t nhi = (t.n + nlo - 1) >> t.bits;
      for (int64_t e = 0; e < nlo; ++e)
        omega64(t.n, e, &tw64[(size_t)(t.lo_off + e) * 2], &tw64[(size_t)(t.lo_off + e) * 2 + 1]);
      for (int64_t e = 0; e < nhi; ++e)
        omega64(t.n, e << t.bits, &tw64[(size_t)(t.hi_off + e) * 2],
                &tw64[(size_t)(t.hi_off + e) * 2 + 1]);
    }
  }
  std::vector<float> tw32;
  const void* tw_host = tw64.data();
  size_t tw_bytes = (size_t)P.tw_elems * P.elem;
  if (P.dtype == PAFC_C64) {
    tw32.resize(tw64.size());
    for (size_t i = 0; i < tw64.size(); ++i) tw32[i] = (float)tw64[i];
    tw_host = tw32.data();
  }
  // index maps (explicit variant and natural-order spectral filters)
  std::vector<int32_t> maps;
  for (auto& ax : P.axes) {
    p->map_off.push_back((int64_t)maps.size());
    maps.insert(maps.end(), ax.pos.begin(), ax.pos.end());
    maps.insert(maps.end(), ax.posinv.begin(), ax.posinv.end());
  }
  hipError_t e = hipMalloc(&p->d_tw, std::max<size_t>(tw_bytes, 16));
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_maps, maps.size() * sizeof(int32_t));
  // the spectrum: N elements, or every slot of the middle pass's tiles when
  // it is stored tile-major (decided below, once the pipelined passes are
  // known); the larger size is reserved either way
  int64_t h_elems = P.N;
  for (size_t i = 0; i < P.conv.size(); ++i)
    if (P.conv[i].kind == 0 && P.conv[i].mid) {
      p->mid_pass = (int)i;
      h_elems = std::max<int64_t>(h_elems, (int64_t)P.conv[i].a.LW * P.conv[i].a.ntiles);
    }
  if (e == hipSuccess) e = hipMalloc(&p->d_H, (size_t)h_elems * P.elem);
  // fault injection (tests of the cleanup path): report the device as full
  // once the first allocations succeeded
  if (e == hipSuccess) {
    const char* f = getenv("PAFC_FAULT_INJECT");
    if (f && strcmp(f, "oom") == 0) e = hipErrorOutOfMemory;
  }
  size_t symtab_bytes = 3;
  for (auto& ax : P.axes) symtab_bytes += (size_t)ax.n;
  symtab_bytes *= 2 * sizeof(double);
  if (e == hipSuccess) e = hipMalloc(&p->d_symtab, symtab_bytes);
  if (e == hipSuccess && P.variant == PAFC_EXPLICIT_PERM)
    e = hipMalloc(&p->d_scratch, (size_t)P.N * P.elem);
  // persistent grids of the pipelined passes: resident blocks per CU x CUs
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess)
      ncu = 0;
    for (auto* seq : {&p->P.conv, &p->P.fwd, &p->P.inv})
      for (Pass& ps : *seq) {
        if (!ps.pipe) continue;
        int nb = ncu > 0 ? pipe_blocks_per_cu(P.dtype == PAFC_C128, ps.pipe_r, ps.pipe_g,
                                              ps.pipe_ng, ps.pipe_kind, ps.pipe_mode,
                                              ps.pipe_threads, ps.pipe_lds, ps.pipe_gm,
                                              ps.pipe_xc)
                         : 0;
        const int64_t want = (int64_t)nb * ncu;
        ps.pipe_grid = (uint32_t)std::min<int64_t>(want, ps.a.ntiles);
        if (nb <= 0) ps.pipe = false;
      }

  }
  // Tile-major spectrum: when the middle pass and the last forward pass (the
  // same piece of the same axis) both run on the pipelined kernel with the
  // same strided tiling, the filter's last forward pass writes the spectrum
  // in the order the middle pass reads it, one contiguous block per tile
  // instead of 16-column row segments (contiguous tiles read whole rows
  // already, and their forward pass stores through LDS).
  if (P.variant == PAFC_PERM_FREE && p->mid_pass >= 0 && !P.fwd.empty() &&
      env_int("PAFC_HTM", 1) != 0) {
    const Pass& m = P.conv[(size_t)p->mid_pass];
    const Pass& f = P.fwd.back();
    const PassArgs &x = m.a, &y = f.a;
    p->h_tm = m.pipe && f.pipe && m.pipe_r == f.pipe_r && m.pipe_g == f.pipe_g &&
              m.pipe_gm == m.pipe_g && f.pipe_gm == f.pipe_g && m.pipe_xc == 0 &&
              f.pipe_xc == 0 &&
              m.pipe_ng == f.pipe_ng && m.pipe_threads == f.pipe_threads &&
              m.pipe_mode == MODE_STRIDED && f.pipe_mode == MODE_STRIDED &&
              x.mode == MODE_STRIDED &&
              y.mode == MODE_STRIDED &&
              x.L == y.L && x.W == y.W && x.S_i == y.S_i && x.S_c == y.S_c && x.S_o == y.S_o &&
              x.ncols == y.ncols && x.tiles_per_slice == y.tiles_per_slice &&
              x.ntiles == y.ntiles &&
              (uint64_t)x.LW * x.ntiles * (uint64_t)P.elem <= 0xFFFFFFFFull;
  }
  // pass descriptors of the three sequences, uploaded once.  Consecutive
  // axis passes walk their tiles in opposite directions, so that a pass
  // starts on the end of the array the previous pass wrote last, which is
  // still in the device's last-level cache when the array is larger
  // than it.
  const bool snake = env_int("PAFC_SNAKE", 1) != 0;
  const bool poison = env_int("PAFC_LDS_POISON", 0) != 0;
  // Streamed reads.  Where the arrays outgrow the device's last-level cache
  // (256 MB Infinity Cache on MI355X), the spectrum is read once per
  // convolution and the sequence's first pass reads the caller's input cold;
  // ordinary loads of either would only evict lines of the array the
  // previous pass wrote, which the current and next passes still read.
  // Non-temporal loads keep those lines (the 256^3 FP64 middle pass 161 ->
  // 130 us, its first pass 101 -> 88 us).  The spectrum is streamed only
  // where each load instruction covers whole 128-byte lines or halves of
  // them (tile-major spectrum, or row segments of 64 bytes or more): with
  // shorter segments the rest of a line is evicted before the tile that
  // needs it reads it (the 2^24 x 2 middle passes, 2-column segments, ran
  // 1.2-1.4x slower streamed).  Smaller arrays keep their spectrum cached
  // across calls and use ordinary loads.
  const int64_t llc = (int64_t)env_int("PAFC_LLC_MB", 256) << 20;
  const int64_t ne = P.N * (int64_t)P.elem;
  p->nt_h = 2 * ne >= llc;
  std::vector<PassArgs> descs;
  for (auto* seq : {&p->P.conv, &p->P.fwd, &p->P.inv}) {
    int i = 0;
    for (Pass& ps : *seq) {
      if (ps.kind != 0) continue;
      ps.desc = (uint32_t)descs.size();
      PassArgs a;
      finalize_args(P, p->d_tw, p->d_H, ps, &a);
      a.rev = snake && (i++ % 2 == 1) ? 1u : 0u;
      a.poison = poison ? 1u : 0u;
      if (p->h_tm && seq == &p->P.conv && &ps == &p->P.conv[(size_t)p->mid_pass]) a.h_tm = 1;
      const int64_t seg = (ps.a.mode == MODE_STRIDED ? (int64_t)ps.a.W : (int64_t)ps.a.L) * P.elem;
      if (ps.mid && 2 * ne >= llc && (a.h_tm || seg >= 64)) a.nt |= 1u;
      if (&ps == &seq->front() && ne >= llc) a.nt |= 2u;
      descs.push_back(a);
    }
  }
  if (p->h_tm && e == hipSuccess)  // staging array of the filter's transform
    e = hipMalloc(&p->d_scratch, (size_t)P.N * P.elem);
  if (p->h_tm) {  // the forward sequence again, its last pass writing tile-major
    p->fwd_tm = p->P.fwd;
    Pass& last = p->fwd_tm.back();
    PassArgs a = descs[last.desc];
    a.tm_store = 1;
    last.desc = (uint32_t)descs.size();
    descs.push_back(a);
  }
  // pafc_convolve_with_filter_noalloc: the middle pass once more, reading
  // the spectrum from this device's `scratch` array (fused permutation-free
  // plans whose spectrum fits the array)
  if (P.variant != PAFC_PERM_FREE || p->mid_pass < 0) {
    p->noalloc_status = PAFC_ERROR_INVALID_VALUE;
  } else if ((uint64_t)h_elems * P.elem > (uint64_t)PAFC_NOALLOC_MAX_BYTES) {
    p->noalloc_status = PAFC_ERROR_UNSUPPORTED_SIZE;
  } else {
    void* addr = nullptr;
    if (scratch_address(p->device, &addr) != hipSuccess) {
      p->noalloc_status = PAFC_ERROR_DEVICE;
    } else {
      p->conv_noalloc = p->P.conv;
      Pass& m = p->conv_noalloc[(size_t)p->mid_pass];
      PassArgs a = descs[m.desc];
      a.H = addr;
      m.desc = (uint32_t)descs.size();
      descs.push_back(a);
      p->noalloc_H = addr;
      p->noalloc_status = PAFC_SUCCESS;
    }
  }
  if (e == hipSuccess)
    e = hipMalloc((void**)&p->d_descs, std::max<size_t>(1, descs.size()) * sizeof(PassArgs));
  if (e != hipSuccess) {
    free_plan(p);
    return from_hip(e);
  }
  e = hipMemcpyAsync(p->d_tw, tw_host, tw_bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->d_maps, maps.data(), maps.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !descs.empty())
    e = hipMemcpyAsync(p->d_descs, descs.data(), descs.size() * sizeof(PassArgs),
                       hipMemcpyHostToDevice, s);
  // the host vectors die here: wait for the copies
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    free_plan(p);
    return from_hip(e);
  }
  p->bytes = tw_bytes + maps.size() * sizeof(int32_t) + descs.size() * sizeof(PassArgs) +
             symtab_bytes +
             (P.variant == PAFC_EXPLICIT_PERM || p->h_tm ? (size_t)P.N * P.elem : 0) +
             (size_t)h_elems * P.elem;
  *out = p;
  return PAFC_SUCCESS;
}

}  // namespace

extern "C" {

pafc_status pafc_plan(pafc_plan_t* out, int ndim, const int64_t* dims, const int* radix,
                      pafc_dtype dtype, pafc_variant variant, void* hip_stream) {
  if (!out) return PAFC_ERROR_INVALID_VALUE;
  *out = nullptr;
  if (variant == PAFC_PRIME_FACTOR || variant == PAFC_PRIME_FACTOR_EXPLICIT)
    return plan_prime_factor(out, ndim, dims, radix, dtype, variant, hip_stream);
  if (is_rader_case(ndim, dims, radix, variant))
    return plan_rader(out, dims[0], dtype, variant, hip_stream);
  if (is_bluestein_case(ndim, dims, radix, variant))
    return plan_bluestein(out, dims[0], dtype, variant, hip_stream);
  return make_plan(out, ndim, dims, radix, dtype, variant, hip_stream, PlanLimits());
}

pafc_status pafc_destroy(pafc_plan_t p) {
  free_plan(p);
  return PAFC_SUCCESS;
}

pafc_status pafc_plan_device_bytes(pafc_plan_t p, size_t* bytes) {
  if (!p || !bytes) return PAFC_ERROR_INVALID_VALUE;
  *bytes = p->bytes;
  return PAFC_SUCCESS;
}

pafc_status pafc_plan_radices(pafc_plan_t p, int axis, int* rho, int* len) {
  if (!p || !rho || !len || axis < 0 || axis >= p->P.ndim || p->inner) return PAFC_ERROR_INVALID_VALUE;
  const auto& r = p->P.axes[(size_t)axis].rho;
  const int cap = *len;
  *len = (int)r.size();
  if (cap < (int)r.size()) return PAFC_ERROR_INVALID_VALUE;
  for (size_t i = 0; i < r.size(); ++i) rho[i] = r[i];
  return PAFC_SUCCESS;
}

// The plan's spectrum from a filter: spatial h -> A^T h by the plan's own
// forward passes; natural-order spectrum -> one reversal pass.  Kept
// unscaled (the 1/N is applied with the product); the explicit variant keeps
// it in natural order, the reversal done here once.
pafc_status load_filter(pafc_plan_t p, const void* h_dev, pafc_filter_domain domain,
                        hipStream_t s) {
  const PlanCore& P = p->P;
  const size_t nbytes = (size_t)P.N * P.elem;
  const bool natural = P.variant == PAFC_EXPLICIT_PERM;
  if (domain == PAFC_FILTER_SPATIAL) {
    if (natural) {
      PAFC_TRY(run_sequence(p, P.fwd, h_dev, p->d_scratch, s));
      PAFC_TRY(run_permute(p, 1, p->d_scratch, p->d_H, nullptr, s));
    } else {
      PAFC_TRY(p->h_tm ? forward_tile_major(p, h_dev, s) : run_sequence(p, P.fwd, h_dev, p->d_H, s));
    }
  } else if (natural) {
    PAFC_TRY(from_hip(hipMemcpyAsync(p->d_H, h_dev, nbytes, hipMemcpyDeviceToDevice, s)));
  } else if (p->h_tm) {  // natural -> digit-reversed -> tile-major, once
    return via_plan_layout(p, s, [&](void* t) { return run_permute(p, 2, h_dev, t, nullptr, s); });
  } else {  // natural -> digit-reversed, once
    PAFC_TRY(run_permute(p, 2, h_dev, p->d_H, nullptr, s));
  }
  return PAFC_SUCCESS;
}

pafc_status pafc_set_filter(pafc_plan_t p, const void* h_dev, pafc_filter_domain domain,
                            void* hip_stream) {
  if (!p || !h_dev || !aligned_for(h_dev, p->P.dtype)) return PAFC_ERROR_INVALID_VALUE;
  if (domain != PAFC_FILTER_SPATIAL && domain != PAFC_FILTER_SPECTRAL_NATURAL)
    return PAFC_ERROR_INVALID_VALUE;
  hipStream_t s = (hipStream_t)hip_stream;
  p->filter_set = false;
  if (is_bluestein(p)) {
    PAFC_TRY(blue_set_filter(p, h_dev, domain, s));
  } else if (is_rader(p)) {
    PAFC_TRY(rader_set_filter(p, h_dev, domain, s));
  } else if (p->inner) {  // reindexed to the grid, then the grid plan's own filter
    PAFC_TRY(pfa_gather(p, h_dev, p->d_scratch, domain == PAFC_FILTER_SPATIAL ? 0 : 1, s));
    PAFC_TRY(pafc_set_filter(p->inner, p->d_scratch, domain, hip_stream));
  } else {
    PAFC_TRY(load_filter(p, h_dev, domain, s));
  }
  p->filter_set = true;
  return PAFC_SUCCESS;
}

pafc_status pafc_convolve_with_filter(pafc_plan_t p, const void* x_dev, const void* h_dev,
                                      void* y_dev, void* hip_stream) {
  if (!p || !x_dev || !h_dev || !y_dev) return PAFC_ERROR_INVALID_VALUE;
  if (!aligned_for(x_dev, p->P.dtype) || !aligned_for(y_dev, p->P.dtype) ||
      !aligned_for(h_dev, p->P.dtype))
    return PAFC_ERROR_INVALID_VALUE;
  hipStream_t s = (hipStream_t)hip_stream;
  if (p->inner) {
    PAFC_TRY(pafc_set_filter(p, h_dev, PAFC_FILTER_SPATIAL, hip_stream));
    return is_bluestein(p) ? blue_convolve(p, x_dev, y_dev, s)
           : is_rader(p)   ? rader_convolve(p, x_dev, y_dev, s)
                           : pfa_convolve(p, x_dev, y_dev, s);
  }
  p->filter_set = false;
  PAFC_TRY(load_filter(p, h_dev, PAFC_FILTER_SPATIAL, s));
  p->filter_set = true;
  return run_sequence(p, p->P.conv, x_dev, y_dev, s);
}

pafc_status pafc_convolve_with_filter_noalloc(pafc_plan_t p, const void* x_dev,
                                              const void* h_dev, void* y_dev,
                                              void* hip_stream) {
  if (!p || !x_dev || !h_dev || !y_dev) return PAFC_ERROR_INVALID_VALUE;
  if (!aligned_for(x_dev, p->P.dtype) || !aligned_for(y_dev, p->P.dtype) ||
      !aligned_for(h_dev, p->P.dtype))
    return PAFC_ERROR_INVALID_VALUE;
  if (p->inner) return PAFC_ERROR_INVALID_VALUE;  // prime-length and prime-factor routes
  if (!p->noalloc_H) return p->noalloc_status;
  hipStream_t s = (hipStream_t)hip_stream;
  void* H = p->noalloc_H;
  // the filter's forward transform into the array (the plan's own spectrum
  // is left as it is); a tile-major spectrum is staged in the plan's
  // staging array and written by the last pass in the middle pass's order
  if (p->h_tm) {
    const void* src = h_dev;
    for (size_t i = 0; i + 1 < p->fwd_tm.size(); ++i) {
      PAFC_TRY(run_pass(p, p->fwd_tm[i], src, p->d_scratch, s));
      src = p->d_scratch;
    }
    PAFC_TRY(run_pass(p, p->fwd_tm.back(), src, H, s));
  } else {
    PAFC_TRY(run_sequence(p, p->P.fwd, h_dev, H, s));
  }
  return run_sequence(p, p->conv_noalloc, x_dev, y_dev, s);
}

pafc_status pafc_set_symbol(pafc_plan_t p, pafc_symbol kind, const double* params, int nparams,
                            void* hip_stream) {
  if (!p || p->inner) return PAFC_ERROR_INVALID_VALUE;  // not for the prime-factor or Bluestein routes
  const PlanCore& P = p->P;
  const int d = P.ndim;
  double t = 0;
  int axis = 0;
  switch (kind) {
    case PAFC_SYMBOL_INV_LAPLACIAN:
    case PAFC_SYMBOL_INV_LAPLACIAN_FD:
      if (nparams != 0) return PAFC_ERROR_INVALID_VALUE;
      break;
    case PAFC_SYMBOL_HEAT:
      if (nparams != 1 || !params || !(params[0] >= 0.0) || !std::isfinite(params[0]))
        return PAFC_ERROR_INVALID_VALUE;
      t = params[0];
      break;
    case PAFC_SYMBOL_DERIVATIVE:
      if (nparams != 1 || !params || params[0] != std::floor(params[0]) || params[0] < 0 ||
          params[0] >= d)
        return PAFC_ERROR_INVALID_VALUE;
      axis = (int)params[0];
      break;
    case PAFC_SYMBOL_GAUSSIAN:
      if (nparams != 1 || !params || !(params[0] >= 0.05) || !(params[0] <= 1e6))
        return PAFC_ERROR_INVALID_VALUE;
      t = params[0];  // sigma
      break;
    default:
      return PAFC_ERROR_INVALID_VALUE;
  }
  // Per-axis tables of the natural frequencies k < n_i, in long double,
  // rounded once to FP64.  kt = k (k <= n/2) or k - n, w = 2 pi kt / n.
  const long double pi = 3.141592653589793238462643383279502884L;
  const int mode = (kind == PAFC_SYMBOL_INV_LAPLACIAN || kind == PAFC_SYMBOL_INV_LAPLACIAN_FD) ? 0 : 1;
  std::vector<double> g;  // (re, im) pairs; axes padded to 3 with one neutral entry
  std::vector<uint32_t> off(3, 0), len(3, 1);
  for (int i = 0; i < 3; ++i) {
    off[(size_t)i] = (uint32_t)(g.size() / 2);
    if (i >= d) {  // a missing axis: one neutral entry
      g.push_back(mode == 0 ? 0.0 : 1.0);
      g.push_back(0.0);
      continue;
    }
    const int64_t n = P.axes[(size_t)i].n;
    len[(size_t)i] = (uint32_t)n;
    // Gaussian: theta(kt) = sum_m exp(-2 pi^2 sigma^2 (kt/n + m)^2) for
    // 0 <= kt <= n/2 (theta is even in kt), the images m and -m added as one
    // pair in order of increasing |m|; terms beyond |m| = M are below
    // exp(-100) of the largest
    std::vector<long double> theta;
    if (kind == PAFC_SYMBOL_GAUSSIAN) {
      const long double c = 2.0L * pi * pi * (long double)t * (long double)t;
      const int64_t M = 2 + (int64_t)std::ceil(std::sqrt(100.0 / (double)c));
      theta.resize((size_t)(n / 2 + 1));
      for (int64_t kt = 0; kt <= n / 2; ++kt) {
        const long double xk = (long double)kt / (long double)n;
        long double sum = expl(-c * xk * xk);
        for (int64_t m = 1; m <= M; ++m) {
          const long double a = xk + (long double)m, b = xk - (long double)m;
          sum += expl(-c * a * a) + expl(-c * b * b);
        }
        theta[(size_t)kt] = sum;
      }
    }
    for (int64_t k = 0; k < n; ++k) {
      const int64_t kt = 2 * k <= n ? k : k - n;
      const long double w = 2.0L * pi * (long double)kt / (long double)n;
      long double re = 0, im = 0;
      if (kind == PAFC_SYMBOL_INV_LAPLACIAN) {
        re = w * w;
      } else if (kind == PAFC_SYMBOL_INV_LAPLACIAN_FD) {
        const int64_t km = std::min<int64_t>(k, n - k);  // sin(pi k / n) = sin(pi (n - k) / n)
        const long double sv = sinl(pi * (long double)km / (long double)n);
        re = 4.0L * sv * sv;
      } else if (kind == PAFC_SYMBOL_HEAT) {
        re = expl(-(long double)t * w * w);
      } else if (kind == PAFC_SYMBOL_GAUSSIAN) {
        re = theta[(size_t)(kt < 0 ? -kt : kt)] / theta[0];
      } else {  // derivative: i w on its axis (0 at the Nyquist frequency), 1 elsewhere
        if (i == axis) {
          im = (2 * k == n) ? 0.0L : w;
        } else {
          re = 1.0L;
        }
      }
      g.push_back((double)re);
      g.push_back((double)im);
    }
  }
  // shape as three axes (leading ones of length 1)
  const int32_t* m[3] = {nullptr, nullptr, nullptr};
  uint32_t nn[3] = {1, 1, 1}, oo[3] = {0, 0, 0};
  const bool natural = P.variant == PAFC_EXPLICIT_PERM;
  for (int i = 0; i < d; ++i) {
    const int slot = 3 - d + i;
    nn[slot] = len[(size_t)i];
    oo[slot] = off[(size_t)i];
    m[slot] = natural ? nullptr : map_ptr(p, i, true);  // position -> frequency
  }
  for (int slot = 0; slot < 3 - d; ++slot) oo[slot] = off[(size_t)(d + slot)];
  hipStream_t s = (hipStream_t)hip_stream;
  p->filter_set = false;
  PAFC_TRY(from_hip(hipMemcpyAsync(p->d_symtab, g.data(), g.size() * sizeof(double),
                                   hipMemcpyHostToDevice, s)));
  auto write = [&](void* H) {
    return from_hip(launch_symbol(P.dtype == PAFC_C128, H, p->d_symtab, m[0], m[1], m[2], nn[0],
                                  nn[1], nn[2], oo[0], oo[1], oo[2], mode, s));
  };
  PAFC_TRY(p->h_tm ? via_plan_layout(p, s, write) : write(p->d_H));
  // the host table dies here: wait for its upload
  PAFC_TRY(from_hip(hipStreamSynchronize(s)));
  p->filter_set = true;
  return PAFC_SUCCESS;
}

pafc_status pafc_convolve(pafc_plan_t p, const void* x_dev, void* y_dev, void* hip_stream) {
  if (!p || !x_dev || !y_dev) return PAFC_ERROR_INVALID_VALUE;
  if (!aligned_for(x_dev, p->P.dtype) || !aligned_for(y_dev, p->P.dtype))
    return PAFC_ERROR_INVALID_VALUE;
  if (!p->filter_set) return PAFC_ERROR_FILTER_NOT_SET;
  if (is_bluestein(p)) return blue_convolve(p, x_dev, y_dev, (hipStream_t)hip_stream);
  if (is_rader(p)) return rader_convolve(p, x_dev, y_dev, (hipStream_t)hip_stream);
  if (p->inner) return pfa_convolve(p, x_dev, y_dev, (hipStream_t)hip_stream);
  return run_sequence(p, p->P.conv, x_dev, y_dev, (hipStream_t)hip_stream);
}

pafc_status pafc_profile_passes(pafc_plan_t p, const void* x_dev, void* y_dev, void* hip_stream,
                                int reps, double* ms_per_pass, int64_t* bytes_per_pass,
                                double* ms_per_rep, int* npass) {
  if (!p || !x_dev || !y_dev || !npass || reps < 1) return PAFC_ERROR_INVALID_VALUE;
  if (!aligned_for(x_dev, p->P.dtype) || !aligned_for(y_dev, p->P.dtype))
    return PAFC_ERROR_INVALID_VALUE;
  if (!p->filter_set) return PAFC_ERROR_FILTER_NOT_SET;
  const int n = route_launches(p);
  const int cap = *npass;
  *npass = n;
  if (cap < n || !ms_per_pass) return PAFC_ERROR_INVALID_VALUE;
  PAFC_TRY(profile_impl(p, x_dev, y_dev, (hipStream_t)hip_stream, reps, -1, ms_per_pass,
                        ms_per_rep, nullptr));
  if (bytes_per_pass)
    for (int k = 0; k < n; ++k) bytes_per_pass[k] = route_pass_bytes(p, k);
  return PAFC_SUCCESS;
}

pafc_status pafc_profile_launch(pafc_plan_t p, const void* x_dev, void* y_dev, void* hip_stream,
                                int reps, int launch, double* ms_launch, double* ms_per_rep) {
  if (!p || !x_dev || !y_dev || !ms_launch || reps < 1) return PAFC_ERROR_INVALID_VALUE;
  if (!aligned_for(x_dev, p->P.dtype) || !aligned_for(y_dev, p->P.dtype))
    return PAFC_ERROR_INVALID_VALUE;
  if (!p->filter_set) return PAFC_ERROR_FILTER_NOT_SET;
  if (launch < 0 || launch >= route_launches(p)) return PAFC_ERROR_INVALID_VALUE;
  return profile_impl(p, x_dev, y_dev, (hipStream_t)hip_stream, reps, launch, nullptr,
                      ms_per_rep, ms_launch);
}

pafc_status pafc_forward(pafc_plan_t p, const void* x_dev, void* z_dev, void* hip_stream) {
  if (!p || !x_dev || !z_dev || p->inner) return PAFC_ERROR_INVALID_VALUE;
  if (!aligned_for(x_dev, p->P.dtype) || !aligned_for(z_dev, p->P.dtype))
    return PAFC_ERROR_INVALID_VALUE;
  return run_sequence(p, p->P.fwd, x_dev, z_dev, (hipStream_t)hip_stream);
}

pafc_status pafc_inverse(pafc_plan_t p, const void* z_dev, void* y_dev, void* hip_stream) {
  if (!p || p->inner || !z_dev || !y_dev) return PAFC_ERROR_INVALID_VALUE;
  if (!aligned_for(z_dev, p->P.dtype) || !aligned_for(y_dev, p->P.dtype))
    return PAFC_ERROR_INVALID_VALUE;
  hipStream_t s = (hipStream_t)hip_stream;
  PAFC_TRY(run_sequence(p, p->P.inv, z_dev, y_dev, s));
  return from_hip(launch_scale(p->P.dtype == PAFC_C128, y_dev, p->P.N, 1.0 / (double)p->P.N, s));
}

pafc_status pafc_twiddle(int64_t n, int64_t e, double* re, double* im) {
  if (n < 1 || !re || !im) return PAFC_ERROR_INVALID_VALUE;
  omega64(n, e, re, im);
  return PAFC_SUCCESS;
}

pafc_status pafc_stream_copy(const void* src_dev, void* dst_dev, size_t bytes, int kind,
                             void* hip_stream) {
  if (!src_dev || !dst_dev || (bytes % 16) != 0 || kind < 0 || kind > 4)
    return PAFC_ERROR_INVALID_VALUE;
  // the tile probes: 256 rows of a multiple of 16 columns, below 2^32 elements
  if (kind >= 3 && (bytes % (256u * 16u * 16u) != 0 || bytes / 16 >= (1ull << 32)))
    return PAFC_ERROR_INVALID_VALUE;
  if (((uintptr_t)src_dev & 15) || ((uintptr_t)dst_dev & 15)) return PAFC_ERROR_INVALID_VALUE;
  return from_hip(launch_stream_copy(kind, src_dev, dst_dev, (int64_t)(bytes / 16),
                                     (hipStream_t)hip_stream));
}

pafc_status pafc_set_tuning(const char* text) {
  std::map<TuneKey, TuneVal> t;
  if (text) {
    const char* c = text;
    while (*c) {
      const char* eol = strchr(c, '\n');
      std::string line(c, eol ? (size_t)(eol - c) : strlen(c));
      c = eol ? eol + 1 : c + strlen(c);
      const size_t h = line.find('#');
      if (h != std::string::npos) line.resize(h);
      if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
      char dt[16];
      long long n = 0, split = 0;
      int W = 0, Wo = 0, g3 = 0, g5 = 0, g3i = 0;
      const int got = sscanf(line.c_str(), "%15s %lld %lld %d %d %d %d %d", dt, &n, &split, &W,
                             &Wo, &g3, &g5, &g3i);
      if (got != 4 && got != 7 && got != 8) return PAFC_ERROR_INVALID_VALUE;
      const int d = !strcmp(dt, "c128") ? PAFC_C128 : !strcmp(dt, "c64") ? PAFC_C64 : -1;
      if (d < 0 || n < 2 || split < 0 || W < 0 || Wo < 0 || g3 < 0 || g3 > 3 || g5 < 0 ||
          g5 > 2 || g3i < 0 || g3i > 3)
        return PAFC_ERROR_INVALID_VALUE;
      TuneVal v;
      v.split = split;
      v.W = W;
      v.Wo = Wo;
      v.gmax3 = g3;
      v.gmax5 = g5;
      v.gmax3i = g3i;
      t[{d, (int64_t)n}] = v;
    }
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.swap(t);
  return PAFC_SUCCESS;
}

}  // extern "C"

// =================================================================== batch

struct pafc_batch_s {
  int form = PAFC_BATCH_PERSISTENT;
  int dtype = PAFC_C128;
  size_t elem = 16;
  int count = 0;
  int nfilters = 0;
  std::vector<int64_t> sizes, offsets;
  std::vector<int> fid;
  int64_t total = 0;
  std::map<int64_t, pafc_plan_t> plans;  // one plan per size class
  std::vector<int64_t> fsize;            // size class of each filter
  std::vector<void*> d_spec;             // per-filter spectra, inside d_spec_all
  std::vector<int64_t> spec_off;         // element offset of each in d_spec_all
  void* d_spec_all = nullptr;
  std::vector<bool> fset;
  PassArgs* d_descs = nullptr;
  BatchTile* d_tiles = nullptr;
  // classes form: per size class, (data offset, spectrum offset) of each of
  // its problems
  uint32_t* d_prob = nullptr;
  // classes form on several streams: each size class's launches form a
  // chain on one stream (0: the caller's; i > 0: aux[i - 1]); the chains
  // fork from the caller's stream and join back into it
  int nstreams = 1;
  std::vector<hipStream_t> aux;
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> join_ev;
  // persistent form: one job per problem, claimed through the control words
  BatchJob* d_jobs = nullptr;
  BatchCtl* d_ctl = nullptr;
  uint32_t njobs = 0;
  struct Level {  // one launch: the tiles of one pass level in one register class
                  // whose LDS needs allow the same number of resident blocks
                  // (levels form), or the whole batch (persistent form)
    int level = 0;
    uint32_t first = 0, count = 0, threads = 64;
    size_t lds = 0;
    int cls = 0;
    int64_t bytes = 0;  // algorithmic HBM bytes of the launch
    bool persist = false;
    uint32_t grid = 0;  // persistent form and pipelined launches: resident blocks
    // classes form: one pipelined launch over every problem of a size class
    bool pipe = false;
    int r = 0, g = 0, ng = 0, kind = 0, mode = 0, gm = 0;
    uint32_t desc = 0;
    int64_t n = 0;   // the class's length (classes form)
    int stream = 0;  // the stream of its class's chain (classes form)
  };
  std::vector<Level> levels;
  std::string desc;
  size_t bytes = 0;
};

namespace {
void free_batch(pafc_batch_t b) {
  if (!b) return;
  for (auto& kv : b->plans) free_plan(kv.second);
  if (b->d_spec_all) (void)hipFree(b->d_spec_all);
  if (b->d_prob) (void)hipFree(b->d_prob);
  for (hipStream_t st : b->aux)
    if (st) (void)hipStreamDestroy(st);
  if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
  for (hipEvent_t e : b->join_ev)
    if (e) (void)hipEventDestroy(e);
  if (b->d_descs) (void)hipFree(b->d_descs);
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  if (b->d_ctl) (void)hipFree(b->d_ctl);
  delete b;
}

hipError_t launch_level(pafc_batch_t b, const pafc_batch_s::Level& L, const void* x, void* y,
                        hipStream_t s) {
  const bool dbl = b->dtype == PAFC_C128;
  if (L.persist)
    return launch_batch_persist(dbl, b->d_descs, b->d_jobs, b->njobs, b->d_ctl, L.grid, L.lds, x,
                                y, s);
  if (L.pipe)
    return launch_pipe_batch(dbl, L.r, L.g, L.ng, L.kind, L.mode, L.gm, b->d_descs + L.desc,
                             L.grid, L.threads, L.lds, L.level == 0 ? x : y, y, s);
  return launch_batch(dbl, L.cls, b->d_descs, b->d_tiles, L.first, L.count, L.level == 0 ? x : y,
                      y, L.threads, L.lds, s);
}

// Limits of the size-class plans of the persistent form: every pass runs in
// one kernel of 256 threads, the register class of groups up to R = 16 (so
// radix-3 groups of at most 2 stages, radix-5 of 1), and one dynamic LDS
// size for the whole launch, which sets the resident blocks per CU: tiles
// are held to PAFC_BATCH_LDS_KB (measured best on the mixed workload: 80 KB
// in FP64, two blocks per CU; 32 KB in FP32, five).  The tuning table's
// entries are measured for the other forms' kernels and are not taken:
// without them the persistent launch measured 2.289 vs 2.328 ms FP64 and
// 1.693 vs 2.363 ms FP32.
PlanLimits persist_limits(int dtype) {
  PlanLimits lim;
  const int kb = env_int("PAFC_BATCH_LDS_KB", dtype == PAFC_C128 ? 80 : 32);
  lim.lds = (size_t)std::max(16, std::min(156, kb)) * 1024;  // below the 159 KB limit
  lim.g3 = 2;
  lim.g5 = 1;
  lim.table = false;
  return lim;
}
}  // namespace

extern "C" {

pafc_status pafc_batch_plan(pafc_batch_t* out, int count, const int64_t* sizes,
                            const int* filter_ids, int nfilters, pafc_dtype dtype,
                            pafc_batch_form form, void* hip_stream) {
  if (!out) return PAFC_ERROR_INVALID_VALUE;
  *out = nullptr;
  if (count < 1 || !sizes || !filter_ids || nfilters < 1) return PAFC_ERROR_INVALID_VALUE;
  if (dtype != PAFC_C64 && dtype != PAFC_C128) return PAFC_ERROR_INVALID_VALUE;
  if (form != PAFC_BATCH_PERSISTENT && form != PAFC_BATCH_LEVELS && form != PAFC_BATCH_AUTO &&
      form != PAFC_BATCH_CLASSES)
    return PAFC_ERROR_INVALID_VALUE;
  // the form measured faster for the element type on the mixed workload
  const bool auto_form = form == PAFC_BATCH_AUTO;
  if (auto_form) form = PAFC_BATCH_CLASSES;
  pafc_batch_t b = new (std::nothrow) pafc_batch_s;
  if (!b) return PAFC_ERROR_OUT_OF_MEMORY;
  b->form = form;
  b->dtype = dtype;
  b->elem = dtype == PAFC_C128 ? 16 : 8;
  b->count = count;
  b->nfilters = nfilters;
  b->fsize.assign((size_t)nfilters, 0);
  b->fset.assign((size_t)nfilters, false);
  b->d_spec.assign((size_t)nfilters, nullptr);
  hipStream_t s = (hipStream_t)hip_stream;
  auto fail = [&](pafc_status st) {
    free_batch(b);
    return st;
  };
  // every argument is checked before any device call; the batched form runs
  // the pass plans of {2,3,5}-smooth lengths only (the prime-length routes
  // have stages of their own)
  for (int i = 0; i < count; ++i) {
    const int64_t n = sizes[i];
    const int f = filter_ids[i];
    if (n < 2 || f < 0 || f >= nfilters) return fail(PAFC_ERROR_INVALID_VALUE);
    if (b->fsize[(size_t)f] != 0 && b->fsize[(size_t)f] != n) return fail(PAFC_ERROR_INVALID_VALUE);
    b->fsize[(size_t)f] = n;
  }
  for (int i = 0; i < count; ++i)
    if (!smooth235(sizes[i])) return fail(PAFC_ERROR_UNSUPPORTED_SIZE);
  for (int i = 0; i < count; ++i) {
    const int64_t n = sizes[i];
    const int f = filter_ids[i];
    b->sizes.push_back(n);
    b->fid.push_back(f);
    b->offsets.push_back(b->total);
    b->total += n;
    if (!b->plans.count(n)) {
      pafc_plan_t p = nullptr;
      PlanLimits lim = form == PAFC_BATCH_PERSISTENT ? persist_limits(dtype) : PlanLimits();
      lim.batched = true;
      pafc_status st = make_plan(&p, 1, &n, nullptr, dtype, PAFC_PERM_FREE, hip_stream, lim);
      if (st != PAFC_SUCCESS) return fail(st);
      b->plans[n] = p;
    }
  }
  // the filter spectra, in one allocation, each 256-byte aligned
  int64_t spec_total = 0;
  b->spec_off.assign((size_t)nfilters, -1);
  for (int f = 0; f < nfilters; ++f) {
    if (b->fsize[(size_t)f] == 0) continue;  // unused filter id
    b->spec_off[(size_t)f] = spec_total;
    const int64_t al = 256 / (int64_t)b->elem;
    spec_total += (b->fsize[(size_t)f] + al - 1) / al * al;
  }
  // the pipelined kernel indexes with 32-bit byte offsets
  const bool fits32 = (uint64_t)b->total * b->elem <= (1ull << 32) &&
                      (uint64_t)spec_total * b->elem <= (1ull << 32);
  if (form == PAFC_BATCH_CLASSES && !fits32) {
    // the levels form has the same size-class plans and no such bound (the
    // persistent form's limits would need other plans)
    if (!auto_form) return fail(PAFC_ERROR_UNSUPPORTED_SIZE);
    form = PAFC_BATCH_LEVELS;
    b->form = form;
  }
  if (hipMalloc(&b->d_spec_all, (size_t)spec_total * b->elem) != hipSuccess)
    return fail(PAFC_ERROR_OUT_OF_MEMORY);
  for (int f = 0; f < nfilters; ++f)
    if (b->spec_off[(size_t)f] >= 0)
      b->d_spec[(size_t)f] = (char*)b->d_spec_all + b->spec_off[(size_t)f] * (int64_t)b->elem;
  // classes form: the problems of each size class in memory order, as
  // (data offset, spectrum offset) pairs
  std::map<int64_t, uint32_t> ptab_first, ptab_count;
  std::vector<uint32_t> ptab;
  if (form == PAFC_BATCH_CLASSES) {
    for (auto& kv : b->plans) {
      const int64_t n = kv.first;
      ptab_first[n] = (uint32_t)ptab.size();
      uint32_t c = 0;
      for (int i = 0; i < count; ++i)
        if (b->sizes[(size_t)i] == n) {
          ptab.push_back((uint32_t)b->offsets[(size_t)i]);
          ptab.push_back((uint32_t)b->spec_off[(size_t)b->fid[(size_t)i]]);
          ++c;
        }
      ptab_count[n] = c;
    }
    if (hipMalloc((void**)&b->d_prob, ptab.size() * sizeof(uint32_t)) != hipSuccess)
      return fail(PAFC_ERROR_OUT_OF_MEMORY);
  }
  // descriptors: one per (filter, pass level)
  std::vector<PassArgs> descs;
  std::map<std::pair<int, int>, uint32_t> didx;
  std::vector<uint32_t> dthreads;
  std::vector<size_t> dlds;
  std::vector<int> dcls;
  for (int f = 0; f < nfilters; ++f) {
    if (b->fsize[(size_t)f] == 0) continue;
    pafc_plan_t p = b->plans[b->fsize[(size_t)f]];
    const auto& conv = p->P.conv;
    for (size_t l = 0; l < conv.size(); ++l) {
      PassArgs a;
      finalize_args(p->P, p->d_tw, b->d_spec[(size_t)f], conv[l], &a);
      a.poison = env_int("PAFC_LDS_POISON", 0) != 0 ? 1u : 0u;
      didx[{f, (int)l}] = (uint32_t)descs.size();
      descs.push_back(a);
      dthreads.push_back(conv[l].threads);
      dlds.push_back(conv[l].lds);
      dcls.push_back(conv[l].cls);
    }
  }
  // classes form: each pass of a size class that its plan runs on the
  // pipelined kernel becomes one launch over every problem of the class
  std::map<std::pair<int64_t, int>, pafc_batch_s::Level> pipe_levels;
  if (form == PAFC_BATCH_CLASSES) {
    int ncu = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu <= 0)
      return fail(PAFC_ERROR_DEVICE);
    const bool dbl = dtype == PAFC_C128;
    for (auto& kv : b->plans) {
      const int64_t n = kv.first;
      const pafc_plan_t pp = kv.second;
      const uint32_t np = ptab_count[n];
      // filters of the class (each read once by the middle pass)
      std::vector<bool> fcls((size_t)nfilters, false);
      int64_t nf = 0;
      for (int i = 0; i < count; ++i)
        if (b->sizes[(size_t)i] == n && !fcls[(size_t)b->fid[(size_t)i]]) {
          fcls[(size_t)b->fid[(size_t)i]] = true;
          ++nf;
        }
      for (size_t l = 0; l < pp->P.conv.size(); ++l) {
        const Pass& ps = pp->P.conv[l];
        if (ps.kind != 0 || !ps.pipe || ps.pipe_grid == 0 || ps.pipe_xc != 0) continue;
        const uint64_t nt = (uint64_t)ps.a.ntiles * np;
        if (np == 0 || nt >= (1ull << 32)) continue;
        const int bpc = pipe_batch_blocks_per_cu(dbl, ps.pipe_r, ps.pipe_g, ps.pipe_ng, ps.pipe_kind,
                                                 ps.pipe_mode, ps.pipe_threads, ps.pipe_lds,
                                                 ps.pipe_gm);
        if (bpc <= 0) continue;  // no batched instance: the general engine runs it
        PassArgs a;
        finalize_args(pp->P, pp->d_tw, b->d_spec_all, ps, &a);
        a.poison = env_int("PAFC_LDS_POISON", 0) != 0 ? 1u : 0u;
        a.tm_store = 0;
        a.prob_off = b->d_prob + ptab_first[n];
        a.tiles_per_prob = a.ntiles;
        a.divProb = make_fastdiv(a.ntiles);
        a.ntiles = (uint32_t)nt;
        pafc_batch_s::Level L;
        L.pipe = true;
        L.level = (int)l;
        L.n = n;
        L.r = ps.pipe_r;
        L.g = ps.pipe_g;
        L.ng = ps.pipe_ng;
        L.kind = ps.pipe_kind;
        L.mode = ps.pipe_mode;
        L.gm = ps.pipe_gm;
        L.desc = (uint32_t)descs.size();
        L.count = (uint32_t)nt;
        L.threads = ps.pipe_threads;
        L.lds = ps.pipe_lds;
        L.grid = (uint32_t)std::min<uint64_t>((uint64_t)bpc * (uint64_t)ncu, nt);
        L.bytes = 2 * n * (int64_t)b->elem * np + (ps.mid ? nf * n * (int64_t)b->elem : 0);
        descs.push_back(a);
        dthreads.push_back(ps.pipe_threads);
        dlds.push_back(ps.pipe_lds);
        dcls.push_back(ps.cls);
        pipe_levels[{n, (int)l}] = L;
      }
    }
  }
  // tiles per (level, register class, LDS occupancy) launch, longest
  // problems first.  The tiles of one level are independent, so splitting a
  // level only lets each part run with its own kernel's register occupancy
  // and with the dynamic LDS of its own largest tile (a launch's LDS size is
  // the maximum over its tiles, and sets how many blocks fit on a CU).
  std::vector<int> order((size_t)count);
  for (int i = 0; i < count; ++i) order[(size_t)i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return b->sizes[(size_t)x] > b->sizes[(size_t)y]; });
  auto blocks_per_cu = [](size_t lds) { return (int)std::min<size_t>(8, kLdsBudget / std::max<size_t>(lds, 1)); };
  std::vector<BatchTile> tiles;
  std::vector<BatchJob> jobs;
  // every pass level of the longest plan (a 1-D plan has 1, 3 or, for
  // lengths cut twice, 5 passes)
  int nlevels = 0;
  for (auto& kv : b->plans) nlevels = std::max(nlevels, (int)kv.second->P.conv.size());
  if (form == PAFC_BATCH_PERSISTENT) {
    // one job per problem, largest first: every pass of its size class, whose
    // descriptors are consecutive from the first one
    pafc_batch_s::Level L;
    L.persist = true;
    L.threads = 256;
    for (size_t d = 0; d < descs.size(); ++d) {
      // the kernel holds the register groups up to R = 16 (class 0; class 2
      // is a subset of it)
      if (dcls[d] == 1) return fail(PAFC_ERROR_UNSUPPORTED_SIZE);
      L.lds = std::max(L.lds, dlds[d]);
    }
    std::vector<bool> fseen((size_t)nfilters, false);
    for (int i : order) {
      const int f = b->fid[(size_t)i];
      const pafc_plan_t pp = b->plans[b->sizes[(size_t)i]];
      const uint32_t d0 = didx.at({f, 0});
      const uint32_t np = (uint32_t)pp->P.conv.size();
      for (uint32_t q = 1; q < np; ++q)
        if (didx.at({f, (int)q}) != d0 + q) return fail(PAFC_ERROR_DEVICE);
      jobs.push_back(BatchJob{d0, np, b->offsets[(size_t)i]});
      L.bytes += 2 * (int64_t)np * b->sizes[(size_t)i] * (int64_t)b->elem;
      if (!fseen[(size_t)f]) {
        fseen[(size_t)f] = true;
        L.bytes += b->sizes[(size_t)i] * (int64_t)b->elem;
      }
    }
    int ncu = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return fail(PAFC_ERROR_DEVICE);
    const int bpc = batch_persist_blocks_per_cu(b->dtype == PAFC_C128, L.lds);
    if (bpc <= 0 || ncu <= 0) return fail(PAFC_ERROR_DEVICE);
    L.grid = (uint32_t)std::min<int64_t>((int64_t)bpc * ncu, (int64_t)jobs.size());
    L.count = (uint32_t)jobs.size();
    b->njobs = (uint32_t)jobs.size();
    b->levels.push_back(L);
    nlevels = 0;  // no level launches
  }
  // classes form on several streams (PAFC_BATCH_STREAMS, default 6: one
  // batch of 4096 problems measured 2.145 / 1.883 / 1.876 / 1.852 / 1.827 /
  // 1.765 / 1.870 ms FP64 and 1.244 / 1.096 / 1.016 / 1.017 / 0.982 / 0.950 /
  // 1.012 ms FP32 on 1 / 2 / 3 / 4 / 5 / 6 / 8 streams): the general engine's
  // launches are made per size class too, so that every launch belongs to
  // one chain
  if (form == PAFC_BATCH_CLASSES)
    b->nstreams = std::max(1, std::min(8, env_int("PAFC_BATCH_STREAMS", 6)));
  std::vector<int64_t> split_classes{0};  // 0: one group over all classes
  if (b->nstreams > 1) {
    split_classes.clear();
    for (auto it = b->plans.rbegin(); it != b->plans.rend(); ++it) split_classes.push_back(it->first);
  }
  for (int l = 0; l < nlevels; ++l) {
    // the level's pipelined launches (classes form), longest classes first,
    // then the general engine's for the rest of the level
    for (auto it = pipe_levels.rbegin(); it != pipe_levels.rend(); ++it)
      if (it->first.second == l) b->levels.push_back(it->second);
    for (int64_t only : split_classes)
    for (int cls = 0; cls < 3; ++cls)
    for (int bpc = 1; bpc <= 8; ++bpc) {
      pafc_batch_s::Level L;
      L.level = l;
      L.cls = cls;
      L.n = only;
      L.first = (uint32_t)tiles.size();
      std::vector<bool> fseen((size_t)nfilters, false);
      for (int i : order) {
        const int f = b->fid[(size_t)i];
        if (only != 0 && b->sizes[(size_t)i] != only) continue;
        if (pipe_levels.count({b->sizes[(size_t)i], l})) continue;
        auto it = didx.find({f, l});
        if (it == didx.end() || dcls[it->second] != cls) continue;
        if (blocks_per_cu(dlds[it->second]) != bpc) continue;
        const PassArgs& a = descs[it->second];
        for (uint32_t t = 0; t < a.ntiles; ++t)
          tiles.push_back(BatchTile{it->second, t, b->offsets[(size_t)i]});
        L.threads = std::max(L.threads, dthreads[it->second]);
        L.lds = std::max(L.lds, dlds[it->second]);
        L.bytes += 2 * b->sizes[(size_t)i] * (int64_t)b->elem;
        const pafc_plan_t pp = b->plans[b->sizes[(size_t)i]];
        if (pp->P.conv[(size_t)l].mid && !fseen[(size_t)f]) {
          fseen[(size_t)f] = true;
          L.bytes += b->sizes[(size_t)i] * (int64_t)b->elem;
        }
      }
      L.count = (uint32_t)tiles.size() - L.first;
      if (L.count) b->levels.push_back(L);
    }
  }
  // chains to streams, longest (in bytes) first onto the least loaded
  // stream; then the streams and the events that fork and join them
  if (b->nstreams > 1) {
    std::map<int64_t, int64_t> load;
    for (const auto& L : b->levels) load[L.n] += L.bytes;
    std::vector<std::pair<int64_t, int64_t>> chains(load.begin(), load.end());
    std::sort(chains.begin(), chains.end(),
              [](const auto& x, const auto& y) { return x.second > y.second; });
    std::vector<int64_t> sl((size_t)b->nstreams, 0);
    std::map<int64_t, int> stream_of;
    for (const auto& c : chains) {
      const int k = (int)(std::min_element(sl.begin(), sl.end()) - sl.begin());
      stream_of[c.first] = k;
      sl[(size_t)k] += c.second;
    }
    for (auto& L : b->levels) L.stream = stream_of[L.n];
    for (int k = 1; k < b->nstreams; ++k) {
      hipStream_t st = nullptr;
      hipEvent_t e = nullptr;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
        return fail(PAFC_ERROR_DEVICE);
      b->aux.push_back(st);
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        return fail(PAFC_ERROR_DEVICE);
      b->join_ev.push_back(e);
    }
    if (hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) != hipSuccess)
      return fail(PAFC_ERROR_DEVICE);
  }
  // every tile's problem must lie inside the packed arrays, and its
  // descriptor must have been built for that problem's length (the filter
  // spectrum it reads has that length)
  {
    std::vector<int64_t> desc_n(descs.size(), 0);
    for (auto& kv : didx) desc_n[kv.second] = b->fsize[(size_t)kv.first.first];
    for (const BatchTile& t : tiles) {
      const int64_t n = desc_n[t.desc];
      if (t.offset < 0 || t.offset + n > b->total || t.tile >= descs[t.desc].ntiles)
        return fail(PAFC_ERROR_INVALID_VALUE);
    }
    for (size_t q = 0; q + 1 < ptab.size(); q += 2)
      if (ptab[q] >= (uint64_t)b->total || ptab[q + 1] >= (uint64_t)spec_total)
        return fail(PAFC_ERROR_INVALID_VALUE);
    for (auto& kv : pipe_levels) {
      const int64_t n = kv.first.first;
      const uint32_t q0 = ptab_first[n], nq = ptab_count[n];
      for (uint32_t q = 0; q < nq; ++q)
        if ((int64_t)ptab[q0 + 2 * q] + n > b->total) return fail(PAFC_ERROR_INVALID_VALUE);
    }
    for (const BatchJob& j : jobs) {
      if (j.npass == 0 || (size_t)j.desc + j.npass > descs.size())
        return fail(PAFC_ERROR_INVALID_VALUE);
      for (uint32_t q = 0; q < j.npass; ++q) {
        const int64_t n = desc_n[j.desc + q];
        if (j.offset < 0 || j.offset + n > b->total || n != desc_n[j.desc])
          return fail(PAFC_ERROR_INVALID_VALUE);
      }
    }
  }
  hipError_t e = hipMalloc((void**)&b->d_descs, descs.size() * sizeof(PassArgs));
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_tiles, std::max<size_t>(1, tiles.size()) * sizeof(BatchTile));
  if (e == hipSuccess && !jobs.empty()) {
    e = hipMalloc((void**)&b->d_jobs, jobs.size() * sizeof(BatchJob));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_ctl, sizeof(BatchCtl));
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->d_jobs, jobs.data(), jobs.size() * sizeof(BatchJob),
                         hipMemcpyHostToDevice, s);
    // zero once here; each launch leaves the control words zero again
    if (e == hipSuccess) e = hipMemsetAsync(b->d_ctl, 0, sizeof(BatchCtl), s);
  }
  if (e == hipSuccess && !ptab.empty())
    e = hipMemcpyAsync(b->d_prob, ptab.data(), ptab.size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_descs, descs.data(), descs.size() * sizeof(PassArgs),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !tiles.empty())
    e = hipMemcpyAsync(b->d_tiles, tiles.data(), tiles.size() * sizeof(BatchTile),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(from_hip(e));
  // description and bytes
  char buf[256];
  snprintf(buf, sizeof(buf),
           "{\"count\": %d, \"total_elems\": %lld, \"size_classes\": %zu, \"form\": \"%s\", "
           "\"streams\": %d, \"levels\": [",
           count, (long long)b->total, b->plans.size(),
           form == PAFC_BATCH_PERSISTENT ? "persistent"
           : form == PAFC_BATCH_CLASSES  ? "classes"
                                         : "levels",
           b->nstreams);
  b->desc = buf;
  for (size_t l = 0; l < b->levels.size(); ++l) {
    auto& L = b->levels[l];
    if (L.persist)
      snprintf(buf, sizeof(buf),
               "%s{\"persistent\": 1, \"jobs\": %u, \"grid\": %u, \"threads\": %u, "
               "\"lds\": %zu}",
               l ? ", " : "", L.count, L.grid, L.threads, L.lds);
    else if (L.pipe)
      snprintf(buf, sizeof(buf),
               "%s{\"level\": %d, \"class\": %lld, \"pipe\": 1, \"tiles\": %u, \"grid\": %u, "
               "\"threads\": %u, \"lds\": %zu, \"stream\": %d}",
               l ? ", " : "", L.level, (long long)L.n, L.count, L.grid, L.threads, L.lds, L.stream);
    else
      snprintf(buf, sizeof(buf),
               "%s{\"level\": %d, \"tiles\": %u, \"threads\": %u, \"lds\": %zu, \"cls\": %d, "
               "\"class\": %lld, \"stream\": %d}",
               l ? ", " : "", L.level, L.count, L.threads, L.lds, L.cls, (long long)L.n, L.stream);
    b->desc += buf;
  }
  b->desc += "], \"plans\": [";
  bool first = true;
  for (auto& kv : b->plans) {
    b->desc += first ? "" : ", ";
    first = false;
    b->desc += describe_core(kv.second->P);
  }
  b->desc += "]}";
  b->bytes = descs.size() * sizeof(PassArgs) + tiles.size() * sizeof(BatchTile) +
             jobs.size() * sizeof(BatchJob) + (jobs.empty() ? 0 : sizeof(BatchCtl)) +
             ptab.size() * sizeof(uint32_t);
  for (auto& kv : b->plans) b->bytes += kv.second->bytes - (size_t)kv.second->P.N * b->elem;
  for (int f = 0; f < nfilters; ++f) b->bytes += (size_t)b->fsize[(size_t)f] * b->elem;
  *out = b;
  return PAFC_SUCCESS;
}

pafc_status pafc_batch_set_filter(pafc_batch_t b, int filter_id, const void* h_dev,
                                  pafc_filter_domain domain, void* hip_stream) {
  if (!b || !h_dev || filter_id < 0 || filter_id >= b->nfilters) return PAFC_ERROR_INVALID_VALUE;
  if (!aligned_for(h_dev, b->dtype)) return PAFC_ERROR_INVALID_VALUE;
  const int64_t n = b->fsize[(size_t)filter_id];
  if (n == 0) return PAFC_ERROR_INVALID_VALUE;
  pafc_plan_t p = b->plans[n];
  hipStream_t s = (hipStream_t)hip_stream;
  void* dst = b->d_spec[(size_t)filter_id];
  if (domain == PAFC_FILTER_SPATIAL) {
    PAFC_TRY(run_sequence(p, p->P.fwd, h_dev, dst, s));
  } else if (domain == PAFC_FILTER_SPECTRAL_NATURAL) {
    PAFC_TRY(run_permute(p, 2, h_dev, dst, nullptr, s));
  } else {
    return PAFC_ERROR_INVALID_VALUE;
  }
  // kept unscaled: the middle op of the size class applies its 1/n
  b->fset[(size_t)filter_id] = true;
  return PAFC_SUCCESS;
}

pafc_status pafc_batch_convolve(pafc_batch_t b, const void* x_dev, void* y_dev, void* hip_stream) {
  if (!b || !x_dev || !y_dev) return PAFC_ERROR_INVALID_VALUE;
  if (!aligned_for(x_dev, b->dtype) || !aligned_for(y_dev, b->dtype)) return PAFC_ERROR_INVALID_VALUE;
  for (int i = 0; i < b->count; ++i)
    if (!b->fset[(size_t)b->fid[(size_t)i]]) return PAFC_ERROR_FILTER_NOT_SET;
  hipStream_t s = (hipStream_t)hip_stream;
  if (b->nstreams > 1) {
    // fork: every chain's stream starts after the caller's prior work
    PAFC_TRY(from_hip(hipEventRecord(b->fork_ev, s)));
    for (hipStream_t st : b->aux) PAFC_TRY(from_hip(hipStreamWaitEvent(st, b->fork_ev, 0)));
  }
  for (auto& L : b->levels)
    PAFC_TRY(from_hip(launch_level(b, L, x_dev, y_dev, L.stream == 0 ? s : b->aux[(size_t)L.stream - 1])));
  if (b->nstreams > 1) {
    // join: the caller's stream continues after every chain
    for (size_t k = 0; k < b->aux.size(); ++k) {
      PAFC_TRY(from_hip(hipEventRecord(b->join_ev[k], b->aux[k])));
      PAFC_TRY(from_hip(hipStreamWaitEvent(s, b->join_ev[k], 0)));
    }
  }
  return PAFC_SUCCESS;
}

pafc_status pafc_batch_profile(pafc_batch_t b, const void* x_dev, void* y_dev, void* hip_stream,
                               int reps, double* ms_per_level, int64_t* bytes_per_level,
                               double* ms_per_rep, int* nlevel) {
  if (!b || !x_dev || !y_dev || !nlevel || reps < 1 || !ms_per_level) return PAFC_ERROR_INVALID_VALUE;
  std::vector<size_t> used;
  for (size_t l = 0; l < b->levels.size(); ++l) used.push_back(l);
  const int n = (int)used.size();
  const int cap = *nlevel;
  *nlevel = n;
  if (cap < n) return PAFC_ERROR_INVALID_VALUE;
  for (int i = 0; i < b->count; ++i)
    if (!b->fset[(size_t)b->fid[(size_t)i]]) return PAFC_ERROR_FILTER_NOT_SET;
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<hipEvent_t> ev((size_t)(n + 1) * reps, nullptr);
  pafc_status st = PAFC_SUCCESS;
  for (auto& e : ev)
    if (st == PAFC_SUCCESS) st = from_hip(timing_event(&e));
  for (int r = 0; r < reps && st == PAFC_SUCCESS; ++r) {
    hipEvent_t* E = ev.data() + (size_t)r * (n + 1);
    st = from_hip(hipEventRecord(E[0], s));
    for (int k = 0; k < n && st == PAFC_SUCCESS; ++k) {
      auto& L = b->levels[used[(size_t)k]];
      st = from_hip(launch_level(b, L, x_dev, y_dev, s));
      if (st == PAFC_SUCCESS) st = from_hip(hipEventRecord(E[k + 1], s));
    }
  }
  if (st == PAFC_SUCCESS) st = from_hip(hipStreamSynchronize(s));
  for (int k = 0; k < n && st == PAFC_SUCCESS; ++k) {
    double tot = 0;
    for (int r = 0; r < reps && st == PAFC_SUCCESS; ++r) {
      float ms = 0;
      st = from_hip(hipEventElapsedTime(&ms, ev[(size_t)r * (n + 1) + k], ev[(size_t)r * (n + 1) + k + 1]));
      tot += ms;
    }
    ms_per_level[k] = tot / reps;
    if (bytes_per_level) bytes_per_level[k] = b->levels[used[(size_t)k]].bytes;
  }
  for (int r = 0; r < reps && ms_per_rep && st == PAFC_SUCCESS; ++r) {
    float ms = 0;
    st = from_hip(hipEventElapsedTime(&ms, ev[(size_t)r * (n + 1)], ev[(size_t)r * (n + 1) + n]));
    ms_per_rep[r] = ms;
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  return st;
}

pafc_status pafc_batch_destroy(pafc_batch_t b) {
  free_batch(b);
  return PAFC_SUCCESS;
}

pafc_status pafc_batch_device_bytes(pafc_batch_t b, size_t* bytes) {
  if (!b || !bytes) return PAFC_ERROR_INVALID_VALUE;
  *bytes = b->bytes;
  return PAFC_SUCCESS;
}

pafc_status pafc_batch_describe(pafc_batch_t b, char* buf, size_t cap, size_t* needed) {
  if (!b) return PAFC_ERROR_INVALID_VALUE;
  if (needed) *needed = b->desc.size() + 1;
  if (buf && cap > 0) {
    size_t n = std::min(cap - 1, b->desc.size());
    memcpy(buf, b->desc.data(), n);
    buf[n] = 0;
  }
  return PAFC_SUCCESS;
}

}  // extern "C"
