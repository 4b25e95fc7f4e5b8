// Host side of the C ABI declared in include/rw.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rw.h"
#include "rw_doe.h"
#include "rw_det.h"
#include "rw_launch.h"

using namespace rw;

namespace {

thread_local std::string g_last_error;

rw_status fail(rw_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(RW_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// Gauss-Legendre nodes/weights on [-1, 1] (Newton on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        break;
      }
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
}

// Arguments a captured launch sequence was recorded with.
struct GraphKey {
  const void* p[10];
  bool operator==(const GraphKey& o) const {
    for (int i = 0; i < 10; ++i)
      if (p[i] != o.p[i]) return false;
    return true;
  }
};
struct GraphState {
  bool valid = false;
  GraphKey key{};
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  void reset() {
    if (x) (void)hipGraphExecDestroy(x);
    if (g) (void)hipGraphDestroy(g);
    x = nullptr;
    g = nullptr;
    valid = false;
  }
};

}  // namespace

struct rw_plan {
  // description
  std::vector<rw_surface> surf;
  rw_doe_desc doe;
  std::vector<rw_param_ref> prm;
  rw_config cfg;
  int n_surf, s_doe, n_pairs, n_lambda, n_field, R, R2, P, M, N, Q, nf, w, H, W;
  size_t n_total;
  bool planar_doe, has_post;
  bool lds_patch;
  int n_class;              // patch classes, largest side first
  int class_p[4], class_m[4];
  bool class_lds[4];
  void* d_tw_cls[4] = {nullptr, nullptr, nullptr, nullptr};   // FFT twiddles per class M
  int doe_blocks;           // workgroups the workspace is sized for (upper bound)
  int ray_block;            // side of the spatial ray blocks (default)
  // launch shape of the ray-wave kernels per direction (rw_autotune may change it)
  int blocks_dir[2];        // [0] forward, [1] backward: persistent workgroups
  int rb_dir[2];            // side of the spatial ray blocks
  int acc_side;             // side of the block-private dL/dt accumulator
  int emit;                 // record slots per ray
  int group_pairs;          // pairs per launch group (memory-bounded)
  bool g2;                  // straight-through gradient of p_mag draws in the backward
  bool tiled_groups;        // several groups, each with room for its interpolated records
                            // (rw_forward_backward interpolates them tile by tile)
  bool tiled_interp;        // one launch group: the backward interpolates the records
                            // of the forward tile by tile
  BinGeom bg;
  int rec_chunk;
  double beta;
  // two-DOE cascade (rw_plan_create_cascade): the fields above describe the
  // second DOE and its incident rays (the first DOE's secondaries); the first
  // DOE's launch grid, map and ray state are these
  const float* cur_phase = nullptr;   // phase map of the forward being enqueued
  bool casc = false;
  int s_doe1 = -1, R1 = 0, R1sq = 0, N1 = 0;
  size_t n1_total = 0;
  DevCfg* d_cfg1 = nullptr;
  size_t off_tmap1 = 0, off_st1 = 0, off_ck1 = 0, off_ctx1 = 0, off_rcls1 = 0;
  size_t off_jdraw1 = 0, off_gt1 = 0, off_gain = 0;   // the cascade's backward
  // device constant tables (owned by the plan)
  DevCfg* d_cfg = nullptr;
  DevPair* d_pairs = nullptr;
  DevSurf* d_base = nullptr;
  DevParam* d_prm = nullptr;
  void* d_tw_nf = nullptr;
  double* d_psi = nullptr;
  double base_sensor_z;
  // workspace layout
  size_t off_live, off_tmap, off_st, off_ck, off_grid, off_t1, off_U, off_alpha, off_lossp,
      off_stats, off_wctr, off_scratch, off_gt, off_raygrad, off_lensg, off_G, off_rpos, off_rval,
      off_spos, off_sval, off_cnt, off_offs, off_cur, off_acc, off_ctx, off_dlist, off_sidx,
      off_scur, off_tpos, off_tval, off_tidx, off_work,
      off_jdraw,
      off_interp, off_g2, off_rcls, off_slices, off_heavy, off_islices, off_iheavy, off_dacc,
      total;
  size_t fwd_bytes;        // workspace of a forward-only pass (a prefix of the layout)
  size_t sz_cf, sz_cg;   // sizeof(C2<Tf>), sizeof(C2<Tg>)
  // state between forward and backward
  bool fwd_done = false;
  bool fwd_full = false;    // the last forward left the backward's state (draws, slots)
  bool fwd_only = false;    // the forward being enqueued writes no backward state
  bool no_alloc = false;    // enqueue without events or graphs (rw_forward_static)
  const float* fwd_target = nullptr;
  const int32_t* fwd_replay = nullptr;
  const float* fwd_phase = nullptr;
  const float* fwd_psf = nullptr;
  const float* fwd_amp = nullptr;
  void* fwd_ws = nullptr;
  hipStream_t fwd_stream = nullptr;
  // captured launch sequences (rw_set_graph)
  bool graph = false;
  bool capturing = false;
  GraphState gfwd, gbwd, gstep;
  hipStream_t cap_st = nullptr;
  // stage timing
  bool prof = false;
  struct Ev { int stage; hipEvent_t a, b; };
  std::vector<Ev> ev_used;
  std::vector<hipEvent_t> ev_pool;
  hipEvent_t ev_get() {
    if (!ev_pool.empty()) { hipEvent_t e = ev_pool.back(); ev_pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
};

namespace {
// Brackets the launches of one stage with events when profiling is on.
struct StageTimer {
  rw_plan* pl;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  StageTimer(rw_plan* p, int s, hipStream_t stream) : pl(p), stage(s), st(stream) {
    if (pl->prof && !pl->capturing && !pl->no_alloc) {
      a = pl->ev_get(); b = pl->ev_get(); (void)hipEventRecord(a, st);
    }
  }
  ~StageTimer() {
    if (a) { (void)hipEventRecord(b, st); pl->ev_used.push_back({stage, a, b}); }
  }
};

// Replays the launch sequence recorded for `key`, recording it first (on the
// plan's own capture stream) when the arguments changed.  The launch goes on
// the caller's stream.
template <class F>
rw_status graph_run(rw_plan* pl, GraphState& gs, const GraphKey& key, hipStream_t st,
                    F enqueue) {
  if (!gs.valid || !(gs.key == key)) {
    gs.reset();
    if (!pl->cap_st) HIPCHK(hipStreamCreateWithFlags(&pl->cap_st, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(pl->cap_st, hipStreamCaptureModeThreadLocal));
    pl->capturing = true;
    const rw_status r = enqueue(pl->cap_st);
    pl->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(pl->cap_st, &g);
    if (r != RW_OK) {
      if (g) (void)hipGraphDestroy(g);
      return r;
    }
    if (e != hipSuccess)
      return fail(RW_ERR_HIP, std::string("stream capture: ") + hipGetErrorString(e));
    gs.g = g;
    const hipError_t ei = hipGraphInstantiate(&gs.x, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      gs.reset();
      return fail(RW_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
    }
    gs.key = key;
    gs.valid = true;
  }
  HIPCHK(hipGraphLaunch(gs.x, st));
  return RW_OK;
}
}  // namespace

// ------------------------------------------------------------ dispatch -----
namespace {

template <class Tg, int NF>
void launch_grid_fwd(rw_plan* pl, void* ws, hipStream_t st, int pair0, int npairs, float* psf) {
  char* b = (char*)ws;
  const int Q = pl->Q;
  const size_t rows = (size_t)npairs * NF;
  hipLaunchKernelGGL((k_grid_rows_fwd<Tg, NF>), dim3((rows + 3) / 4), dim3(256), 0, st,
                     (const C2<Tg>*)(b + pl->off_grid), (C2<Tg>*)(b + pl->off_t1),
                     (const C2<Tg>*)pl->d_tw_nf, Q, pair0, npairs);
  const size_t cols = (size_t)npairs * Q;
  hipLaunchKernelGGL((k_grid_cols_fwd<Tg, NF>), dim3((cols + 3) / 4), dim3(256), 0, st,
                     (const C2<Tg>*)(b + pl->off_t1), (const C2<Tg>*)pl->d_tw_nf, pl->d_psi, Q,
                     pair0, npairs, (C2<Tg>*)(b + pl->off_U), psf);
}

template <class Tg>
rw_status grid_fwd_t(rw_plan* pl, void* ws, hipStream_t st, int pair0, int npairs, float* psf) {
  switch (pl->nf) {
    case 64: launch_grid_fwd<Tg, 64>(pl, ws, st, pair0, npairs, psf); break;
    case 128: launch_grid_fwd<Tg, 128>(pl, ws, st, pair0, npairs, psf); break;
    case 256: launch_grid_fwd<Tg, 256>(pl, ws, st, pair0, npairs, psf); break;
    case 512: launch_grid_fwd<Tg, 512>(pl, ws, st, pair0, npairs, psf); break;
    case 1024: launch_grid_fwd<Tg, 1024>(pl, ws, st, pair0, npairs, psf); break;
    case 2048: launch_grid_fwd<Tg, 2048>(pl, ws, st, pair0, npairs, psf); break;
    default: return fail(RW_ERR_SHAPE, "unsupported grid size");
  }
  HIPCHK(hipGetLastError());
  return RW_OK;
}

rw_status grid_fwd(rw_plan* pl, void* ws, hipStream_t st, int pair0, int npairs, float* psf) {
  if (pl->cfg.precision == RW_PREC_FP64) return grid_fwd_t<double>(pl, ws, st, pair0, npairs, psf);
  return grid_fwd_t<float>(pl, ws, st, pair0, npairs, psf);
}

DoeArgs doe_args(rw_plan* pl, void* ws, const int32_t* replay, int32_t* idx_out) {
  char* b = (char*)ws;
  DoeArgs a;
  memset(&a, 0, sizeof(a));
  a.cfg = pl->d_cfg;
  a.pairs = pl->d_pairs;
  a.live = (const DevLive*)(b + pl->off_live);
  a.st = (const double*)(b + pl->off_st);
  a.n_total = pl->n_total;
  a.tmap = b + pl->off_tmap;
  a.tw = pl->d_tw_cls[0];
  a.grid = b + pl->off_grid;
  a.rec_pos = b + pl->off_rpos;
  a.rec_val = b + pl->off_rval;
  a.emit = pl->emit;
  a.scratch = pl->lds_patch ? nullptr : b + pl->off_scratch;
  a.replay = replay;
  a.idx_out = idx_out;
  a.stats = (unsigned long long*)(b + pl->off_stats);
  a.wctr = (unsigned long long*)(b + pl->off_wctr);
  a.gt = b + pl->off_gt;
  a.raygrad = (double*)(b + pl->off_raygrad);
  a.lensg = (double*)(b + pl->off_lensg);
  a.acc = b + pl->off_acc;
  a.acc_side = pl->acc_side;
  a.ctx = (RayCtx*)(b + pl->off_ctx);
  a.dlist = b + pl->off_dlist;
  a.ray_class = (unsigned char*)(b + pl->off_rcls);
  a.jdraw = pl->cfg.sampling == RW_SAMPLE_FULL || pl->fwd_only ? nullptr
                                                                 : (int32_t*)(b + pl->off_jdraw);
  a.full = pl->cfg.sampling == RW_SAMPLE_FULL;
  a.cls = 0;
  a.phase = pl->cur_phase;
  return a;
}

template <class T>
void zero(void* p, size_t n, hipStream_t st);

// Ray-wave interface over whole blocks of rays (persistent workgroups).
// R: side of the launch grid of the rays (the plan's, or the first DOE's of a cascade).
rw_status doe_launch(rw_plan* pl, bool fwd, const DoeArgs& a, int pair0, int npairs,
                     hipStream_t st, int R = -1) {
  if (R < 0) R = pl->R;
  RayBlockIter it;
  it.rb = pl->rb_dir[fwd ? 0 : 1];
  it.nbx = (R + it.rb - 1) / it.rb;
  it.per_pair = it.nbx * it.nbx;
  it.R = R;
  const long long n_items = (long long)npairs * it.per_pair;
  // XCD chunks: one contiguous eighth over 8 or more pairs (each eighth holds
  // whole pairs, hence every patch class in like measure); below that, 32
  // chunks per XCD, so that the rays of a class, which cluster in space, reach
  // every XCD
  it.chunk = npairs >= 8 ? (n_items + 7) / 8 : std::max<long long>(1, (n_items + 255) / 256);
  const int blocks = (int)std::min<long long>(n_items, pl->blocks_dir[fwd ? 0 : 1]);
  // one launch per patch class, each over the whole work list (rays of other
  // classes are skipped; dead rays belong to class 0)
  for (int c = 0; c < pl->n_class; ++c) {
    DoeArgs ac = a;
    ac.cls = c;
    zero<unsigned long long>(ac.wctr, 8, st);   // the work-item counters
    ac.tw = pl->d_tw_cls[c];
    const int M = pl->class_m[c];
    const bool lds = pl->class_lds[c];
    bool ok = true;
    hipError_t e;
    switch (pl->cfg.precision) {
      case RW_PREC_FP64:
        e = launch_doe_fp64(fwd, M, lds, ac, it, n_items, pair0, blocks, st, &ok);
        break;
      case RW_PREC_MIXED:
        e = launch_doe_mixed(fwd, M, lds, ac, it, n_items, pair0, blocks, st, &ok);
        break;
      default:
        e = launch_doe_fp32(fwd, M, lds, ac, it, n_items, pair0, blocks, st, &ok);
    }
    if (!ok) return fail(RW_ERR_SHAPE, "unsupported FFT size M for this precision");
    if (e != hipSuccess)
      return fail(RW_ERR_HIP, std::string("DOE kernel launch: ") + hipGetErrorString(e));
  }
  return RW_OK;
}

template <class Tg, int NF>
void launch_grid_bwd(rw_plan* pl, void* ws, hipStream_t st, int pair0, int npairs,
                     const float* dpsf) {
  char* b = (char*)ws;
  const int Q = pl->Q;
  const size_t nq = (size_t)npairs * Q * Q;
  hipLaunchKernelGGL((k_psf_cograd<Tg>), dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st,
                     dpsf, (const float*)pl->fwd_psf, pl->fwd_target,
                     (const double*)(b + pl->off_alpha), (const C2<Tg>*)(b + pl->off_U),
                     pl->d_psi, Q, pair0, npairs, (C2<Tg>*)(b + pl->off_G));
  const size_t cols = (size_t)npairs * Q;
  hipLaunchKernelGGL((k_grid_cols_bwd<Tg, NF>), dim3((unsigned)((cols + 3) / 4)), dim3(256), 0,
                     st, (const C2<Tg>*)(b + pl->off_G), (const C2<Tg>*)pl->d_tw_nf, Q, pair0,
                     npairs, (C2<Tg>*)(b + pl->off_t1));
  const size_t rows = (size_t)npairs * NF;
  hipLaunchKernelGGL((k_grid_rows_bwd<Tg, NF>), dim3((unsigned)((rows + 3) / 4)), dim3(256), 0,
                     st, (const C2<Tg>*)(b + pl->off_t1), (const C2<Tg>*)pl->d_tw_nf, Q, pair0,
                     npairs, (C2<Tg>*)(b + pl->off_grid));
}

template <class Tg>
rw_status grid_bwd_t(rw_plan* pl, void* ws, hipStream_t st, int pair0, int npairs,
                     const float* dpsf) {
  switch (pl->nf) {
    case 64: launch_grid_bwd<Tg, 64>(pl, ws, st, pair0, npairs, dpsf); break;
    case 128: launch_grid_bwd<Tg, 128>(pl, ws, st, pair0, npairs, dpsf); break;
    case 256: launch_grid_bwd<Tg, 256>(pl, ws, st, pair0, npairs, dpsf); break;
    case 512: launch_grid_bwd<Tg, 512>(pl, ws, st, pair0, npairs, dpsf); break;
    case 1024: launch_grid_bwd<Tg, 1024>(pl, ws, st, pair0, npairs, dpsf); break;
    case 2048: launch_grid_bwd<Tg, 2048>(pl, ws, st, pair0, npairs, dpsf); break;
    default: return fail(RW_ERR_SHAPE, "unsupported grid size");
  }
  HIPCHK(hipGetLastError());
  return RW_OK;
}

rw_status grid_bwd(rw_plan* pl, void* ws, hipStream_t st, int pair0, int npairs,
                   const float* dpsf) {
  if (pl->cfg.precision == RW_PREC_FP64) return grid_bwd_t<double>(pl, ws, st, pair0, npairs, dpsf);
  return grid_bwd_t<float>(pl, ws, st, pair0, npairs, dpsf);
}

template <class T>
void zero(void* p, size_t n, hipStream_t st);

// Deterministic mode: the binned records of the group spread as fixed-point
// integers by sub-tiles (LDS, then the group's integer grid), then converted
// into the group's grids.  Byte offsets in the mode's buffer: the bound word,
// the heavy-slice count, the integer grids, the slices per sub-tile, the list.
struct DetLayout {
  size_t grids, slices, heavy, total;
};
static DetLayout det_layout(const BinGeom& g, int group_pairs) {
  const size_t tb = (size_t)det_tb(g), ns = (g.nb / tb) * (g.nb / tb) * group_pairs;
  DetLayout d;
  d.grids = 512;
  d.slices = d.grids + align256((size_t)group_pairs * g.nf * g.nf * 2 * sizeof(long long));
  d.heavy = d.slices + align256(ns);
  d.total = d.heavy + ns * (kDetSlices - 1) * sizeof(uint2);
  return d;
}

template <class Tg>
rw_status det_spread_t(rw_plan* pl, void* ws, hipStream_t st, int pair0, int npairs) {
  char* b = (char*)ws;
  const BinGeom g = pl->bg;
  const size_t per_pair = (size_t)pl->R2 * pl->emit;
  const size_t n = per_pair * (size_t)npairs;
  const size_t ncells = (size_t)npairs * pl->nf * pl->nf;
  const DetLayout dl = det_layout(g, pl->group_pairs);
  char* d0 = b + pl->off_dacc;
  unsigned long long* amax = (unsigned long long*)d0;
  unsigned int* nh = (unsigned int*)(d0 + 256);
  unsigned long long* acc = (unsigned long long*)(d0 + dl.grids);
  unsigned char* sl = (unsigned char*)(d0 + dl.slices);
  uint2* hv = (uint2*)(d0 + dl.heavy);
  const int tb = det_tb(g), side = tb * g.bin, ns = (g.nb / tb) * (g.nb / tb);
  auto blocks = [](size_t m) {
    return dim3((unsigned)std::max<size_t>(1, std::min<size_t>((m + 255) / 256, 16384)));
  };
  StageTimer ts_(pl, RW_STAGE_SPREAD, st);
  zero<unsigned long long>(amax, 1, st);
  zero<unsigned int>(nh, 1, st);
  zero<unsigned long long>(acc, 2 * ncells, st);
  hipLaunchKernelGGL(k_det_absmax<Tg>, blocks(n), dim3(256), 0, st,
                     (const void*)(b + pl->off_rval), n, amax);
  const unsigned long long target = std::max<unsigned long long>(kSpreadTarget, n / 1024);
  const unsigned long long* so = (const unsigned long long*)(b + pl->off_offs);
  hipLaunchKernelGGL(k_det_slices, blocks((size_t)npairs * ns), dim3(256), 0, st, so, g, pair0,
                     npairs, target, sl, hv, nh);
  const void* sp = (const void*)(b + pl->off_spos);
  const void* sv = (const void*)(b + pl->off_sval);
  const size_t lds = (size_t)side * side * 2 * sizeof(unsigned long long);
  const dim3 sg(ns, npairs), hg(1024);
  const unsigned long long* am = amax;
  switch (pl->w) {
#define RW_DET_CASE(W)                                                                        \
    case W:                                                                                   \
      hipLaunchKernelGGL((k_det_tiles<Tg, W>), sg, dim3(256), lds, st, sp, sv, so, g,         \
                         pl->beta, pair0, n, am, acc, (const unsigned char*)sl,               \
                         (const uint2*)nullptr, (const unsigned int*)nullptr);                \
      hipLaunchKernelGGL((k_det_tiles<Tg, W>), hg, dim3(256), lds, st, sp, sv, so, g,         \
                         pl->beta, pair0, n, am, acc, (const unsigned char*)sl,               \
                         (const uint2*)hv, (const unsigned int*)nh);                          \
      break;
    RW_DET_CASE(4) RW_DET_CASE(5) RW_DET_CASE(6) RW_DET_CASE(7) RW_DET_CASE(8)
    RW_DET_CASE(9) RW_DET_CASE(10) RW_DET_CASE(11) RW_DET_CASE(12)
    RW_DET_CASE(13) RW_DET_CASE(14) RW_DET_CASE(15) RW_DET_CASE(16)
#undef RW_DET_CASE
    default: return fail(RW_ERR_SHAPE, "spread_width must be in [4, 16]");
  }
  hipLaunchKernelGGL(k_det_store<Tg>, blocks(ncells), dim3(256), 0, st,
                     (const unsigned long long*)acc, ncells, n, am,
                     (C2<Tg>*)(b + pl->off_grid) + (size_t)pair0 * pl->nf * pl->nf);
  HIPCHK(hipGetLastError());
  return RW_OK;
}

template <class Tg>
rw_status bin_and_spread_t(rw_plan* pl, void* ws, hipStream_t st, int pair0, int npairs) {
  char* b = (char*)ws;
  const BinGeom g = pl->bg;
  const size_t per_pair = (size_t)pl->R2 * pl->emit;
  const int chunk = pl->rec_chunk;
  const dim3 grid((unsigned)((per_pair + chunk - 1) / chunk), (unsigned)npairs);
  unsigned int* cnt = (unsigned int*)(b + pl->off_cnt) + (size_t)pair0 * g.keys;
  unsigned long long* offs = (unsigned long long*)(b + pl->off_offs) + (size_t)pair0 * g.keys;
  unsigned long long* cur = (unsigned long long*)(b + pl->off_cur) + (size_t)pair0 * g.keys;
  StageTimer* tb_ = new StageTimer(pl, RW_STAGE_BIN, st);
  zero<unsigned int>(cnt, (size_t)npairs * g.keys, st);
  hipLaunchKernelGGL(k_rec_hist<Tg>, grid, dim3(256), g.keys * sizeof(unsigned int), st,
                     (const void*)(b + pl->off_rpos), (const void*)(b + pl->off_rval), per_pair,
                     chunk, g, pair0, (unsigned int*)(b + pl->off_cnt));
  const int fpc = 1 << (2 * g.sshift);
  const int nsup = g.keys / fpc;
  constexpr int C = RecChunk<Tg>::C;
  unsigned long long* scur = (unsigned long long*)(b + pl->off_scur) + (size_t)pair0 * nsup;
  unsigned int* work = (unsigned int*)(b + pl->off_work);
  hipLaunchKernelGGL(k_rec_scan, dim3(1), dim3(1024), 0, st, (const unsigned int*)cnt,
                     (size_t)npairs * g.keys, fpc, C, offs, cur, scur, work);
  const bool slots = (pl->tiled_interp || pl->tiled_groups) && !pl->fwd_only;   // record slots
  unsigned int* tidx = slots ? (unsigned int*)(b + pl->off_tidx) : nullptr;
  const unsigned long long* offs_all = (const unsigned long long*)(b + pl->off_offs);
  hipLaunchKernelGGL((k_rec_place<Tg, true>), dim3((unsigned)((per_pair + C - 1) / C), npairs),
                     dim3(256), 0, st, (const void*)(b + pl->off_rpos),
                     (const void*)(b + pl->off_rval), (const unsigned int*)nullptr, per_pair,
                     offs_all, (const unsigned int*)work, g, pair0,
                     (unsigned long long*)(b + pl->off_scur), (void*)(b + pl->off_tpos),
                     (void*)(b + pl->off_tval), tidx);
  // every super-bin takes ceil(count / C) workgroups: at most records / C + super-bins
  const size_t nitems = (size_t)npairs * nsup;
  hipLaunchKernelGGL((k_rec_place<Tg, false>),
                     dim3((unsigned)((size_t)npairs * per_pair / C + nitems)), dim3(256), 0, st,
                     (const void*)(b + pl->off_tpos), (const void*)(b + pl->off_tval),
                     (const unsigned int*)tidx, nitems, offs_all, (const unsigned int*)work, g,
                     pair0, (unsigned long long*)(b + pl->off_cur), (void*)(b + pl->off_spos),
                     (void*)(b + pl->off_sval),
                     slots ? (unsigned int*)(b + pl->off_sidx) : nullptr);
  delete tb_;
  if (pl->cfg.deterministic) return det_spread_t<Tg>(pl, ws, st, pair0, npairs);
  const int tile = 4 * g.bin;
  const int ntiles = (g.nf / tile) * (g.nf / tile);
  StageTimer ts_(pl, RW_STAGE_SPREAD, st);
  const dim3 sg(ntiles, npairs);
  const size_t lds = (size_t)tile * (tile + pl->w) * sizeof(C2<Tg>);
  const void* sp = (const void*)(b + pl->off_spos);
  const void* sv = (const void*)(b + pl->off_sval);
  const unsigned long long* so = (const unsigned long long*)(b + pl->off_offs);
  C2<Tg>* gr = (C2<Tg>*)(b + pl->off_grid);
  // heavy tiles (records concentrated by a focusing system) in slices
  unsigned char* sl = (unsigned char*)(b + pl->off_slices);
  unsigned int* nh = (unsigned int*)(b + pl->off_heavy);
  uint2* hv = (uint2*)(b + pl->off_heavy + 256);
  zero<unsigned int>(nh, 1, st);
  // a slice is at least kSpreadTarget records and about 1/1024 of the group's
  const unsigned long long target =
      std::max<unsigned long long>(kSpreadTarget, (unsigned long long)npairs * per_pair / 1024);
  hipLaunchKernelGGL(k_spread_slices, dim3((unsigned)(((size_t)npairs * ntiles + 255) / 256)),
                     dim3(256), 0, st, so, g, pair0, npairs, target, sl, hv, nh);
  const dim3 hg(1024);
  switch (pl->w) {
#define RW_SPREAD_CASE(W)                                                                     \
    case W:                                                                                   \
      hipLaunchKernelGGL((k_spread_tiles<Tg, W>), sg, dim3(256), lds, st, sp, sv, so, g,      \
                         pl->beta, pair0, gr, (const unsigned char*)sl, (const uint2*)nullptr, \
                         (const unsigned int*)nullptr);                                       \
      hipLaunchKernelGGL((k_spread_tiles<Tg, W>), hg, dim3(256), lds, st, sp, sv, so, g,      \
                         pl->beta, pair0, gr, (const unsigned char*)sl, (const uint2*)hv,      \
                         (const unsigned int*)nh);                                            \
      break;
    RW_SPREAD_CASE(4) RW_SPREAD_CASE(5) RW_SPREAD_CASE(6) RW_SPREAD_CASE(7) RW_SPREAD_CASE(8)
    RW_SPREAD_CASE(9) RW_SPREAD_CASE(10) RW_SPREAD_CASE(11) RW_SPREAD_CASE(12)
    RW_SPREAD_CASE(13) RW_SPREAD_CASE(14) RW_SPREAD_CASE(15) RW_SPREAD_CASE(16)
#undef RW_SPREAD_CASE
    default: return fail(RW_ERR_SHAPE, "spread_width must be in [4, 16]");
  }
  HIPCHK(hipGetLastError());
  return RW_OK;
}

// Type-2 interpolation of the sensor-grid cogradient at every record of the
// forward, tile by tile (backward, one launch group only).
template <class Tg>
rw_status interp_tiles_t(rw_plan* pl, void* ws, hipStream_t st, int pair0, int npairs) {
  char* b = (char*)ws;
  const BinGeom g = pl->bg;
  const int nsb = g.nb / 2;
  const dim3 grid((unsigned)(nsb * nsb), (unsigned)npairs);
  const size_t lds = (size_t)interp_side(g.bin, pl->w) * interp_side(g.bin, pl->w) * sizeof(C2<Tg>);
  StageTimer ti_(pl, RW_STAGE_INTERP, st);
  const void* sp = (const void*)(b + pl->off_spos);
  const unsigned int* si = (const unsigned int*)(b + pl->off_sidx);
  const unsigned long long* so = (const unsigned long long*)(b + pl->off_offs);
  const C2<Tg>* adj = (const C2<Tg>*)(b + pl->off_grid);
  C2<Tg>* out = (C2<Tg>*)(b + pl->off_interp);
  // blocks whose records a focusing system has concentrated, in slices
  unsigned char* sl = (unsigned char*)(b + pl->off_islices);
  unsigned int* nh = (unsigned int*)(b + pl->off_iheavy);
  uint2* hv = (uint2*)(b + pl->off_iheavy + 256);
  const size_t per_pair = (size_t)pl->R2 * pl->emit;
  const unsigned long long target =
      std::max<unsigned long long>(16384, (unsigned long long)npairs * per_pair / 2048);
  zero<unsigned int>(nh, 1, st);
  hipLaunchKernelGGL(k_interp_slices, dim3((unsigned)(((size_t)npairs * nsb * nsb + 255) / 256)),
                     dim3(256), 0, st, so, g, pair0, npairs, target, sl, hv, nh);
  const dim3 hg(1024);
  switch (pl->w) {
#define RW_INTERP_CASE(W)                                                                     \
    case W:                                                                                   \
      hipLaunchKernelGGL((k_interp_tiles<Tg, W>), grid, dim3(256), lds, st, sp, si, so, g,   \
                         pl->beta, pair0, adj, out, (const unsigned char*)sl,                 \
                         (const uint2*)nullptr, (const unsigned int*)nullptr);                \
      hipLaunchKernelGGL((k_interp_tiles<Tg, W>), hg, dim3(256), lds, st, sp, si, so, g,     \
                         pl->beta, pair0, adj, out, (const unsigned char*)sl, (const uint2*)hv,\
                         (const unsigned int*)nh);                                            \
      break;
    RW_INTERP_CASE(4) RW_INTERP_CASE(5) RW_INTERP_CASE(6) RW_INTERP_CASE(7) RW_INTERP_CASE(8)
    RW_INTERP_CASE(9) RW_INTERP_CASE(10) RW_INTERP_CASE(11) RW_INTERP_CASE(12)
    RW_INTERP_CASE(13) RW_INTERP_CASE(14) RW_INTERP_CASE(15) RW_INTERP_CASE(16)
#undef RW_INTERP_CASE
    default: return fail(RW_ERR_SHAPE, "spread_width must be in [4, 16]");
  }
  HIPCHK(hipGetLastError());
  return RW_OK;
}

rw_status interp_tiles(rw_plan* pl, void* ws, hipStream_t st, int pair0, int npairs) {
  if (pl->cfg.precision == RW_PREC_FP64) return interp_tiles_t<double>(pl, ws, st, pair0, npairs);
  return interp_tiles_t<float>(pl, ws, st, pair0, npairs);
}

rw_status bin_and_spread(rw_plan* pl, void* ws, hipStream_t st, int pair0, int npairs) {
  if (pl->cfg.precision == RW_PREC_FP64) return bin_and_spread_t<double>(pl, ws, st, pair0, npairs);
  return bin_and_spread_t<float>(pl, ws, st, pair0, npairs);
}

template <class T>
void zero(void* p, size_t n, hipStream_t st) {
  const size_t blocks = std::min<size_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_zero<T>, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, (T*)p, n);
}

}  // namespace

// ----------------------------------------------------------------- API ----
extern "C" {

const char* rw_status_string(rw_status s) {
  switch (s) {
    case RW_OK: return "ok";
    case RW_ERR_INVALID_ARG: return "invalid argument";
    case RW_ERR_SHAPE: return "unsupported shape";
    case RW_ERR_STATE: return "invalid state";
    case RW_ERR_NONFINITE: return "non-finite input";
    case RW_ERR_OOM: return "out of memory";
    case RW_ERR_HIP: return "HIP runtime error";
    case RW_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* rw_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace {
// The first DOE of a two-DOE cascade, as rw_plan_create_cascade hands it to the
// plan builder (which sees the second DOE as the plan's DOE).
struct CascSpec {
  int s1;                 // surface of the first DOE
  rw_doe_desc doe1;
  int R1;                 // launch grid side
  int n1;                 // side of each ray's block of relayed secondaries
  int N1;                 // relayed secondaries per ray (n1^2)
};

rw_status plan_create(const rw_surface* surfaces, int n_surf, const rw_doe_desc* doe,
                      const rw_param_ref* params, int n_params, const rw_config* cfg,
                      const CascSpec* cs, rw_plan** out) {
  if (!surfaces || !doe || !cfg || !out || (n_params > 0 && !params))
    return fail(RW_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (n_surf < 1 || n_surf > RW_MAX_SURF)
    return fail(RW_ERR_SHAPE, "n_surf must be in [1, 8]");
  if (!cfg->lambda_host || !cfg->field_tan_host || !cfg->launch_center_host ||
      !cfg->psf_center_host)
    return fail(RW_ERR_INVALID_ARG, "null host array in config");
  int s_doe = -1;
  for (int s = 0; s < n_surf; ++s)
    if (surfaces[s].carries_doe) {
      if (s_doe >= 0) return fail(RW_ERR_UNSUPPORTED, "more than one DOE surface");
      s_doe = s;
    }
  if (s_doe < 0) return fail(RW_ERR_INVALID_ARG, "no surface carries the DOE");
  for (int i = 0; i < n_params; ++i) {
    if (params[i].surface < 0 || params[i].surface >= n_surf || params[i].field < 0 ||
        params[i].field > RW_PARAM_GAP)
      return fail(RW_ERR_INVALID_ARG, "bad lens parameter reference");
  }
  const int P = cfg->patch_p, pad = cfg->pad_factor;
  const int M = P * pad;
  if (P < 1 || pad < 1 || !is_pow2(M) || M < 16 || M > 256)
    return fail(RW_ERR_SHAPE, "M = pad_factor * patch_p must be a power of two in [16, 256]");
  if (cfg->psf_q < 32 || !is_pow2(cfg->psf_q) || cfg->psf_q > 1024)
    return fail(RW_ERR_SHAPE, "psf_q must be a power of two in [32, 1024]");
  if (cfg->rays_side < 1 || cfg->n_lambda < 1 || cfg->n_field < 1)
    return fail(RW_ERR_SHAPE, "empty ray grid, wavelength or field list");
  if (cfg->sampling < 0 || cfg->sampling > 2 || cfg->precision < 0 || cfg->precision > 2)
    return fail(RW_ERR_INVALID_ARG, "bad sampling or precision");
  if (cfg->grad != RW_GRAD_G1 && cfg->grad != RW_GRAD_G2 && cfg->grad != RW_GRAD_G1_DETACH)
    return fail(RW_ERR_INVALID_ARG, "bad gradient mode");
  if (cfg->grad == RW_GRAD_G2 && !(cfg->tau > 0.0))
    return fail(RW_ERR_INVALID_ARG, "the G2 temperature must be positive");
  if (cfg->sampling != RW_SAMPLE_FULL && (cfg->n_ssr < 1 || cfg->n_ssr > 2048))
    return fail(RW_ERR_SHAPE, "n_ssr must be in [1, 2048]");
  if (doe->H < 1 || doe->W < 1 || !(doe->pitch > 0))
    return fail(RW_ERR_SHAPE, "bad DOE map description");
  if (doe->field != RW_FIELD_AMP_PHASE && doe->field != RW_FIELD_TWO_PHASE)
    return fail(RW_ERR_INVALID_ARG, "bad DOE field mode");
  if (doe->reflective && s_doe != n_surf - 1)
    return fail(RW_ERR_UNSUPPORTED, "a reflective DOE must be the last surface");
  if (cfg->precision == RW_PREC_FP64 && M > 128)
    return fail(RW_ERR_UNSUPPORTED, "FP64 supports M <= 128");
  if (cfg->n_patch_class < 0 || cfg->n_patch_class > 3)
    return fail(RW_ERR_INVALID_ARG, "at most three patch classes besides patch_p");
  for (int i = 0; i < cfg->n_patch_class; ++i) {
    const int q = cfg->patch_class_p[i], mq = q * pad;
    if (q < 1 || q >= (i ? cfg->patch_class_p[i - 1] : P) || !is_pow2(mq) || mq < 16)
      return fail(RW_ERR_SHAPE, "patch classes must be decreasing sides below patch_p whose "
                                "M = pad_factor * side is a power of two >= 16");
  }
  if (cfg->n_patch_class > 0 && !(cfg->curv_eps > 0.0))
    return fail(RW_ERR_INVALID_ARG, "curv_eps must be positive");
  if (cfg->class_draws && (cfg->n_patch_class == 0 || cfg->sampling == RW_SAMPLE_FULL))
    return fail(RW_ERR_INVALID_ARG, "class_draws needs patch classes and MAG or UNI sampling");
  if (!(cfg->bandwidth_periods >= 0.0) || std::isinf(cfg->bandwidth_periods))
    return fail(RW_ERR_INVALID_ARG, "bandwidth_periods must be finite and >= 0");
  if (cfg->bandwidth_periods > 0.0 &&
      (cfg->n_patch_class == 0 || doe->field != RW_FIELD_AMP_PHASE || doe->H < 3 || doe->W < 3))
    return fail(RW_ERR_INVALID_ARG, "adaptive patch sizing needs patch classes, the amplitude-"
                                    "phase field and a map of at least 3 x 3 pixels");
  for (int l = 0; l < cfg->n_lambda; ++l)
    if (!(cfg->lambda_host[l] > 0)) return fail(RW_ERR_INVALID_ARG, "wavelength must be > 0");

  rw_plan* pl = new rw_plan();
  pl->surf.assign(surfaces, surfaces + n_surf);
  pl->doe = *doe;
  pl->prm.assign(params, params + n_params);
  pl->cfg = *cfg;
  pl->n_surf = n_surf;
  pl->s_doe = s_doe;
  pl->n_lambda = cfg->n_lambda;
  pl->n_field = cfg->n_field;
  pl->n_pairs = cfg->n_lambda * cfg->n_field;
  pl->R = cfg->rays_side;
  pl->R2 = cfg->rays_side * cfg->rays_side;
  pl->n_total = (size_t)pl->n_pairs * pl->R2;
  pl->P = P;
  pl->M = M;
  pl->n_class = 1 + cfg->n_patch_class;
  pl->class_p[0] = P;
  for (int i = 0; i < cfg->n_patch_class; ++i) pl->class_p[1 + i] = cfg->patch_class_p[i];
  for (int i = 0; i < pl->n_class; ++i) pl->class_m[i] = pl->class_p[i] * pad;
  pl->N = cfg->sampling == RW_SAMPLE_FULL ? M * M : cfg->n_ssr;
  pl->Q = cfg->psf_q;
  pl->nf = std::max(2 * cfg->psf_q, 64);
  pl->w = cfg->spread_width > 0 ? cfg->spread_width
                                : (cfg->precision == RW_PREC_FP64 ? 13 : 7);
  if (pl->w < 4 || pl->w > 16) {
    delete pl;
    return fail(RW_ERR_SHAPE, "spread_width must be in [4, 16]");
  }
  const double sigma = (double)pl->nf / pl->Q;
  pl->beta = 0.98 * M_PI * pl->w * (1.0 - 0.5 / sigma);
  pl->H = doe->H;
  pl->W = doe->W;
  pl->planar_doe = surfaces[s_doe].curvature == 0.0 && surfaces[s_doe].conic == 0.0 &&
                   surfaces[s_doe].asph[0] == 0.0 && surfaces[s_doe].asph[1] == 0.0 &&
                   surfaces[s_doe].asph[2] == 0.0 && surfaces[s_doe].asph[3] == 0.0 &&
                   !(surfaces[s_doe].gauss_width > 0.0);
  for (int i = 0; i < n_params; ++i)
    if (params[i].surface == s_doe && params[i].field != RW_PARAM_GAP) pl->planar_doe = false;
  pl->has_post = s_doe + 1 < n_surf;
  // G2 differs from G1 only for p ~ |U~|
  pl->g2 = cfg->grad == RW_GRAD_G2 && cfg->sampling == RW_SAMPLE_MAG;
  if (pl->g2 && pl->has_post) {
    delete pl;
    return fail(RW_ERR_UNSUPPORTED, "the G2 gradient needs the sensor directly after the DOE");
  }
  pl->base_sensor_z = cfg->sensor_z;
  const bool dbl_f = cfg->precision == RW_PREC_FP64;
  const bool dbl_g = cfg->precision == RW_PREC_FP64;
  pl->sz_cf = dbl_f ? 16 : 8;
  pl->sz_cg = dbl_g ? 16 : 8;
  // the patch buffer sits in LDS up to M = 128 (float spectra) or M = 64
  // (double spectra), as the precision units instantiate the DOE kernels
  auto in_lds = [&](int m) { return m <= (dbl_f ? 64 : 128); };
  pl->lds_patch = in_lds(M);
  // 8 x 8-ray blocks; 4 x 4 over few pairs, where the items of one class launch
  // (patch classes cluster in space) are too few to balance the workgroups
  pl->ray_block = pl->n_pairs < 8 ? 4 : 8;
  pl->acc_side = 256;
  // several workgroups per CU fit from M = 64 down
  pl->doe_blocks = M <= 64 ? 2048 : 1024;
  pl->blocks_dir[0] = pl->blocks_dir[1] = M <= 64 ? 1024 : 512;
  pl->rb_dir[0] = pl->rb_dir[1] = pl->ray_block;
  for (int i = 0; i < pl->n_class; ++i) pl->class_lds[i] = in_lds(pl->class_m[i]);
  pl->emit = cfg->sampling == RW_SAMPLE_FULL ? M * M : cfg->n_ssr;
  {
    const int nb = std::min(64, pl->nf / 8);
    int shift = 0;
    while ((1 << shift) < pl->nf / nb) ++shift;
    int ss = 0;                                   // super-bins of up to 8 x 8 bins
    while (ss < 3 && (2 << ss) <= nb) ++ss;
    pl->bg = {pl->nf, 1 << shift, shift, nb, nb * nb, ss};
    const size_t tile = 4 * (size_t)pl->bg.bin;
    if (tile * (tile + pl->w) * pl->sz_cg + spread_static_lds(pl->sz_cg / 2, pl->w) > 160 * 1024 ||
        pl->w > 2 * pl->bg.bin) {
      delete pl;
      return fail(RW_ERR_UNSUPPORTED, "PSF size too large for this precision");
    }
  }
  pl->rec_chunk = 16384;
  {
    // launch groups of whole pairs whose secondary-ray records (as produced, after
    // the super-bin pass and sorted) fit in 96 GiB; when all pairs fit in one
    // group with the tiled interpolation's per-record indices (32-bit) and
    // results as well, the backward uses that path
    const size_t nrec_pair = (size_t)pl->R2 * pl->emit;
    const size_t rec_bytes = nrec_pair * 3 * (pl->sz_cg + (dbl_g ? 16 : 8));
    const size_t tiled_bytes = rec_bytes + nrec_pair * (4 + 4 + kInterpStride * pl->sz_cg);
    const size_t budget = cfg->record_budget_bytes ? (size_t)cfg->record_budget_bytes
                                                   : (size_t)96 << 30;
    pl->tiled_interp = cfg->batched && tiled_bytes * pl->n_pairs <= budget &&
                       nrec_pair * pl->n_pairs < ((size_t)1 << 32);
    size_t gp = std::max<size_t>(1, budget / std::max<size_t>(rec_bytes, 1));
    // otherwise groups sized so that each holds its slots and interpolated
    // records too: rw_forward_backward interpolates every group tile by tile
    pl->tiled_groups = false;
    if (!pl->tiled_interp && cfg->batched && tiled_bytes <= budget) {
      gp = std::min(budget / tiled_bytes, (((size_t)1 << 32) - 1) / nrec_pair);
      pl->tiled_groups = gp >= 1;
      gp = std::max<size_t>(gp, 1);
    }
    pl->group_pairs = (int)std::min<size_t>(gp, (size_t)pl->n_pairs);
    if (!cfg->batched) pl->group_pairs = 1;
    if (pl->tiled_interp) pl->group_pairs = pl->n_pairs;
  }

  // host copies of the constant tables
  DevCfg dc;
  memset(&dc, 0, sizeof(dc));
  dc.n_surf = n_surf; dc.s_doe = s_doe; dc.n_pairs = pl->n_pairs; dc.n_field = pl->n_field;
  dc.R = pl->R; dc.R2 = pl->R2; dc.P = P; dc.M = M; dc.N = pl->N; dc.Q = pl->Q; dc.nf = pl->nf;
  dc.w = pl->w; dc.sampling = cfg->sampling; dc.H = doe->H; dc.W = doe->W;
  dc.n_params = n_params;
  dc.pitch = doe->pitch; dc.x0 = doe->x0; dc.y0 = doe->y0;
  dc.inv_pitch = 1.0 / doe->pitch;
  dc.grad = cfg->grad;
  dc.pad = pad;
  dc.n_class = pl->n_class;
  for (int i = 0; i < pl->n_class; ++i) {
    dc.class_p[i] = pl->class_p[i];
    // draws per ray: N, or N (P_k / P_0)^2 (at least one) with class_draws
    const long long nk = (long long)pl->N * pl->class_p[i] * pl->class_p[i] /
                         ((long long)pl->class_p[0] * pl->class_p[0]);
    dc.class_n[i] = cfg->class_draws ? (int)std::max(1LL, nk) : pl->N;
  }
  dc.curv_eps = cfg->curv_eps;
  dc.bw_k2 = cfg->bandwidth_periods > 0.0
                 ? (2.0 * M_PI * cfg->bandwidth_periods) * (2.0 * M_PI * cfg->bandwidth_periods)
                 : 0.0;
  dc.tau = cfg->tau > 0.0 ? cfg->tau : 1.0;
  dc.planar = pl->planar_doe ? 1 : 0;
  dc.reflective = doe->reflective ? 1 : 0;
  dc.ns_idx = doe->reflective ? s_doe : n_surf;
  dc.launch_z = cfg->launch_z; dc.launch_half = cfg->launch_half; dc.psf_pitch = cfg->psf_pitch;
  dc.beta = pl->beta;
  dc.key0 = (uint32_t)(cfg->seed & 0xffffffffu);
  dc.key1 = (uint32_t)(cfg->seed >> 32);
  dc.relay_n1 = 0;
  DevCfg dc1 = dc;
  if (cs) {
    if (!pl->class_lds[0]) {
      delete pl;
      return fail(RW_ERR_UNSUPPORTED, "a DOE cascade needs M <= 128 (FP32, MIXED) or M <= 64 (FP64)");
    }
    const rw_surface& q = surfaces[cs->s1];
    bool planar1 = q.curvature == 0.0 && q.conic == 0.0 && q.asph[0] == 0.0 &&
                   q.asph[1] == 0.0 && q.asph[2] == 0.0 && q.asph[3] == 0.0 &&
                   !(q.gauss_width > 0.0);
    for (int i = 0; i < n_params; ++i)
      if (params[i].surface == cs->s1 && params[i].field != RW_PARAM_GAP) planar1 = false;
    pl->casc = true;
    pl->s_doe1 = cs->s1;
    pl->R1 = cs->R1;
    pl->R1sq = cs->R1 * cs->R1;
    pl->N1 = cs->N1;
    pl->n1_total = (size_t)pl->n_pairs * pl->R1sq;
    dc1.s_doe = cs->s1;
    dc1.R = cs->R1;
    dc1.R2 = pl->R1sq;
    dc1.N = cs->N1;
    dc1.class_n[0] = cs->N1;
    dc1.pitch = cs->doe1.pitch; dc1.x0 = cs->doe1.x0; dc1.y0 = cs->doe1.y0;
    dc1.inv_pitch = 1.0 / cs->doe1.pitch;
    dc1.planar = planar1 ? 1 : 0;
    dc1.relay_n1 = cs->n1;
  }

  std::vector<DevPair> pairs(pl->n_pairs);
  for (int l = 0; l < pl->n_lambda; ++l)
    for (int f = 0; f < pl->n_field; ++f) {
      DevPair& p = pairs[l * pl->n_field + f];
      memset(&p, 0, sizeof(p));
      const double lam = cfg->lambda_host[l];
      p.lam = lam;
      p.k0 = 2.0 * M_PI / lam;
      const double tx = cfg->field_tan_host[2 * f], ty = cfg->field_tan_host[2 * f + 1];
      const double nn = std::sqrt(tx * tx + ty * ty + 1.0);
      p.dir[0] = tx / nn; p.dir[1] = ty / nn; p.dir[2] = 1.0 / nn;
      p.lc[0] = cfg->launch_center_host[2 * f];
      p.lc[1] = cfg->launch_center_host[2 * f + 1];
      p.pc[0] = cfg->psf_center_host[2 * (l * pl->n_field + f)];
      p.pc[1] = cfg->psf_center_host[2 * (l * pl->n_field + f) + 1];
      const double lum = lam * 1e3;
      p.n_med[0] = 1.0;
      for (int s = 0; s < n_surf; ++s)
        p.n_med[s + 1] = surfaces[s].n_A + surfaces[s].n_B / (lum * lum);
    }
  std::vector<DevSurf> base(n_surf);
  for (int s = 0; s < n_surf; ++s) {
    const rw_surface& q = surfaces[s];
    base[s] = {q.z_vertex, q.curvature, q.conic, q.asph[0], q.asph[1], q.asph[2], q.asph[3],
               q.semi_aperture, q.kind, q.carries_doe,
               q.gauss_width > 0.0 ? q.gauss_height : 0.0,
               q.gauss_width > 0.0 ? q.gauss_width : 0.0};
  }
  std::vector<DevParam> prm(std::max(n_params, 1));
  for (int i = 0; i < n_params; ++i) prm[i] = {params[i].surface, params[i].field, params[i].scale};
  // FFT twiddles exp(-2 pi i m / n)
  auto twiddles = [](int n, bool dbl) {
    std::vector<char> out(n * (dbl ? 16 : 8));
    for (int m = 0; m < n; ++m) {
      const double a = -2.0 * M_PI * m / n;
      if (dbl) {
        double v[2] = {std::cos(a), std::sin(a)};
        memcpy(out.data() + m * 16, v, 16);
      } else {
        float v[2] = {(float)std::cos(a), (float)std::sin(a)};
        memcpy(out.data() + m * 8, v, 8);
      }
    }
    return out;
  };
  std::vector<char> twn = twiddles(pl->nf, dbl_g);
  // Fourier transform of the spreading kernel at the kept modes (deconvolution)
  std::vector<double> gx, gw, psi(pl->Q);
  gauss_legendre(200, gx, gw);
  for (int c = 0; c < pl->Q; ++c) {
    const int k = c - pl->Q / 2;
    double s = 0;
    for (size_t i = 0; i < gx.size(); ++i) {
      const double z = 0.5 * pl->w * gx[i];
      const double ph = std::exp(pl->beta * (std::sqrt(1.0 - gx[i] * gx[i]) - 1.0));
      s += gw[i] * 0.5 * pl->w * ph * std::cos(2.0 * M_PI * k * z / pl->nf);
    }
    psi[c] = s;
  }

  {
    // the spreading tile of the largest grids needs more than the default 64 KiB of LDS
    hipError_t ea = hipSuccess, eb = hipSuccess;
#define RW_ATTR(W)                                                                              \
    if (ea == hipSuccess)                                                                       \
      ea = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spread_tiles<float, W>),        \
                               hipFuncAttributeMaxDynamicSharedMemorySize,                     \
                               (int)(160 * 1024 - spread_static_lds(sizeof(float), W)));        \
    if (eb == hipSuccess)                                                                       \
      eb = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spread_tiles<double, W>),       \
                               hipFuncAttributeMaxDynamicSharedMemorySize,                     \
                               (int)(160 * 1024 - spread_static_lds(sizeof(double), W)));       \
    if (ea == hipSuccess)                                                                       \
      ea = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_interp_tiles<float, W>),        \
                               hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);         \
    if (eb == hipSuccess)                                                                       \
      eb = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_interp_tiles<double, W>),       \
                               hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);         \
    if (ea == hipSuccess)                                                                       \
      ea = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_det_tiles<float, W>),           \
                               hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);          \
    if (eb == hipSuccess)                                                                       \
      eb = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_det_tiles<double, W>),          \
                               hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    RW_ATTR(4) RW_ATTR(5) RW_ATTR(6) RW_ATTR(7) RW_ATTR(8) RW_ATTR(9) RW_ATTR(10) RW_ATTR(11)
    RW_ATTR(12) RW_ATTR(13) RW_ATTR(14) RW_ATTR(15) RW_ATTR(16)
#undef RW_ATTR
    if (ea != hipSuccess || eb != hipSuccess) {
      delete pl;
      return fail(RW_ERR_HIP, "hipFuncSetAttribute(MaxDynamicSharedMemorySize) failed");
    }
  }
  auto up = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(dst, bytes);
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = up((void**)&pl->d_cfg, &dc, sizeof(dc));
  if (e == hipSuccess && cs) e = up((void**)&pl->d_cfg1, &dc1, sizeof(dc1));
  if (e == hipSuccess) e = up((void**)&pl->d_pairs, pairs.data(), pairs.size() * sizeof(DevPair));
  if (e == hipSuccess) e = up((void**)&pl->d_base, base.data(), base.size() * sizeof(DevSurf));
  if (e == hipSuccess) e = up((void**)&pl->d_prm, prm.data(), prm.size() * sizeof(DevParam));
  for (int i = 0; i < pl->n_class && e == hipSuccess; ++i) {
    const std::vector<char> twc = twiddles(pl->class_m[i], dbl_f);
    e = up(&pl->d_tw_cls[i], twc.data(), twc.size());
  }
  if (e == hipSuccess) e = up(&pl->d_tw_nf, twn.data(), twn.size());
  if (e == hipSuccess) e = up((void**)&pl->d_psi, psi.data(), psi.size() * sizeof(double));
  if (e != hipSuccess) {
    rw_plan_destroy(pl);
    return fail(e == hipErrorOutOfMemory ? RW_ERR_OOM : RW_ERR_HIP,
                std::string("plan tables: ") + hipGetErrorString(e));
  }

  // workspace layout: what a forward needs first, then the state a forward
  // leaves for the backward (the draws, the records' slots), then the
  // backward's own buffers; a workspace of fwd_bytes runs forward-only passes
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t r = o; o = align256(o + bytes); return r; };
  const size_t nt = pl->n_total;
  const size_t nrec = (size_t)pl->group_pairs * pl->R2 * pl->emit;
  const size_t psz = dbl_g ? 16 : 8;
  const size_t nk = (size_t)pl->n_pairs * pl->bg.keys;
  pl->off_live = take(sizeof(DevLive));
  pl->off_tmap = take((size_t)doe->H * doe->W * pl->sz_cf);
  // a cascade's second DOE also keeps each incident ray's complex amplitude
  pl->off_st = take((cs ? 10 : 8) * nt * sizeof(double));
  pl->off_ck = take((size_t)(s_doe + 1) * 8 * nt * sizeof(double));
  pl->off_grid = take((size_t)pl->n_pairs * pl->nf * pl->nf * pl->sz_cg);
  pl->off_t1 = take((size_t)pl->n_pairs * pl->Q * pl->nf * pl->sz_cg);
  pl->off_U = take((size_t)pl->n_pairs * pl->Q * pl->Q * pl->sz_cg);
  pl->off_alpha = take(pl->n_pairs * sizeof(double));
  pl->off_lossp = take(pl->n_pairs * sizeof(double));
  pl->off_stats = take(RW_N_STATS * sizeof(unsigned long long));
  pl->off_wctr = take(8 * sizeof(unsigned long long));
  pl->off_scratch =
      take(pl->lds_patch ? 0 : (size_t)pl->doe_blocks * doe_buf_elems(M) * pl->sz_cf);
  pl->off_ctx = take((size_t)nt * sizeof(RayCtx));
  pl->off_rcls = take((size_t)nt);
  pl->off_rpos = take(nrec * psz);
  pl->off_rval = take(nrec * pl->sz_cg);
  pl->off_tpos = take(nrec * psz);
  pl->off_tval = take(nrec * pl->sz_cg);
  pl->off_spos = take(nrec * psz);
  pl->off_sval = take(nrec * pl->sz_cg);
  pl->off_scur = take((size_t)pl->n_pairs * (pl->bg.keys >> (2 * pl->bg.sshift)) * 8);
  pl->off_work = take(((size_t)pl->n_pairs * (pl->bg.keys >> (2 * pl->bg.sshift)) + 1) * 4);
  pl->off_cnt = take(nk * sizeof(unsigned int));
  pl->off_offs = take((nk + 1) * sizeof(unsigned long long));
  pl->off_cur = take(nk * sizeof(unsigned long long));
  {
    // slices of the spreading tiles of one launch group, and the list of the
    // heavy tiles' further slices (its length first)
    const int tile = 4 * pl->bg.bin;
    const size_t nt = (size_t)(pl->nf / tile) * (pl->nf / tile) * pl->group_pairs;
    pl->off_slices = take(nt);
    pl->off_heavy = take(256 + nt * (kSpreadSlices - 1) * sizeof(uint2));
  }
  // deterministic mode: its bound and slice count, the group's grids as (re, im)
  // int64, and its slices
  pl->off_dacc = take(cfg->deterministic ? det_layout(pl->bg, pl->group_pairs).total : 0);
  if (cs) {
    // the first DOE: its map, launched rays (state, checkpoints, contexts, classes)
    const size_t n1t = pl->n1_total;
    pl->off_tmap1 = take((size_t)doe->H * doe->W * pl->sz_cf);
    pl->off_st1 = take(8 * n1t * sizeof(double));
    pl->off_ck1 = take((size_t)(cs->s1 + 1) * 8 * n1t * sizeof(double));
    pl->off_ctx1 = take(n1t * sizeof(RayCtx));
    pl->off_rcls1 = take(n1t);
  }
  pl->fwd_bytes = o;
  const size_t bw = 1;
  // state of the forward that only the backward reads
  pl->off_jdraw = take(bw * (cfg->sampling == RW_SAMPLE_FULL ? 0 : (size_t)nt * pl->N * sizeof(int32_t)));
  const bool tl = pl->tiled_interp || pl->tiled_groups;
  pl->off_tidx = take(bw * (tl ? nrec * 4 : 0));
  pl->off_sidx = take(bw * (tl ? nrec * 4 : 0));
  // the backward's own buffers
  pl->off_acc = take(bw * (size_t)pl->doe_blocks * pl->acc_side * pl->acc_side * pl->sz_cg);
  pl->off_g2 = take(bw * (pl->g2 ? (size_t)pl->doe_blocks * ((size_t)pl->N * kG2Rec + (size_t)M * M) *
                                       sizeof(float)
                                 : 0));
  pl->off_dlist = take(bw * (cfg->sampling == RW_SAMPLE_FULL
                                 ? 0 : (size_t)pl->doe_blocks * pl->N * 2 * pl->sz_cf));
  pl->off_gt = take(bw * (size_t)doe->H * doe->W * pl->sz_cg);
  pl->off_raygrad = take(bw * (size_t)RW_RAYGRAD * nt * sizeof(double));
  pl->off_lensg = take(bw * RW_LENSG_SLOTS * sizeof(double));
  pl->off_G = take(bw * (size_t)pl->n_pairs * pl->Q * pl->Q * pl->sz_cg);
  pl->off_interp = take(bw * (tl ? nrec * kInterpStride * pl->sz_cg : 0));
  {
    // slices of the tiled interpolation's blocks (2 x 2 bins) and the list of the
    // heavy blocks' further slices (its length first)
    const size_t nb2 = (size_t)(pl->bg.nb / 2) * (pl->bg.nb / 2) * pl->group_pairs;
    pl->off_islices = take(tl ? nb2 : 0);
    pl->off_iheavy = take(tl ? 256 + nb2 * (kInterpSlices - 1) * sizeof(uint2) : 0);
  }
  if (cs) {
    // the first DOE's draws (left by the forward), its dL/dt, and the second
    // DOE's dL/d(incident amplitude) per ray
    pl->off_jdraw1 = take(cfg->sampling == RW_SAMPLE_FULL ? 0 : pl->n1_total * cs->N1 * sizeof(int32_t));
    pl->off_gt1 = take((size_t)doe->H * doe->W * pl->sz_cg);
    pl->off_gain = take(2 * nt * sizeof(double));
  }
  pl->total = o;
  *out = pl;
  return RW_OK;
}
}  // namespace

extern "C" {

rw_status rw_plan_create(const rw_surface* surfaces, int n_surf, const rw_doe_desc* doe,
                         const rw_param_ref* params, int n_params, const rw_config* cfg,
                         rw_plan** out) {
  return plan_create(surfaces, n_surf, doe, params, n_params, cfg, nullptr, out);
}

rw_status rw_plan_create_cascade(const rw_surface* surfaces, int n_surf, const rw_doe_desc* doe1,
                                 const rw_doe_desc* doe2, int n_ssr2, const rw_param_ref* params,
                                 int n_params, const rw_config* cfg, rw_plan** out) {
  if (!surfaces || !doe1 || !doe2 || !cfg || !out || (n_params > 0 && !params))
    return fail(RW_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (n_surf < 2 || n_surf > RW_MAX_SURF)
    return fail(RW_ERR_SHAPE, "a cascade needs n_surf in [2, 8]");
  int s1 = -1, s2 = -1;
  for (int s = 0; s < n_surf; ++s)
    if (surfaces[s].carries_doe) {
      if (s1 < 0) s1 = s;
      else if (s2 < 0) s2 = s;
      else return fail(RW_ERR_UNSUPPORTED, "more than two DOE surfaces");
    }
  if (s2 < 0) return fail(RW_ERR_INVALID_ARG, "a cascade needs two surfaces that carry a DOE");
  if (doe1->H != doe2->H || doe1->W != doe2->W || doe1->H < 1 || doe1->W < 1 ||
      !(doe1->pitch > 0))
    return fail(RW_ERR_SHAPE, "the two DOE maps must have the same H and W");
  if (doe1->reflective || doe2->reflective)
    return fail(RW_ERR_UNSUPPORTED, "a cascade of reflective DOEs is not built");
  if (doe1->field != doe2->field)
    return fail(RW_ERR_INVALID_ARG, "the two DOEs must share the field mode");
  if (cfg->n_patch_class != 0)
    return fail(RW_ERR_UNSUPPORTED, "a cascade takes one patch class");
  if (cfg->grad == RW_GRAD_G2)
    return fail(RW_ERR_UNSUPPORTED, "the G2 gradient of a cascade is not built");
  const int M = cfg->patch_p * cfg->pad_factor;
  int n1 = 0;
  if (cfg->sampling == RW_SAMPLE_FULL) {
    n1 = M;
  } else {
    while ((n1 + 1) * (n1 + 1) <= cfg->n_ssr) ++n1;
    if (cfg->n_ssr < 1 || n1 * n1 != cfg->n_ssr)
      return fail(RW_ERR_SHAPE, "a cascade needs n_ssr = n1^2 draws at the first DOE");
  }
  if (cfg->sampling != RW_SAMPLE_FULL && (n_ssr2 < 1 || n_ssr2 > 2048))
    return fail(RW_ERR_SHAPE, "n_ssr2 must be in [1, 2048]");
  if (cfg->rays_side < 1 || (long long)cfg->rays_side * n1 > 32768)
    return fail(RW_ERR_SHAPE, "the second DOE's ray grid side rays_side * n1 exceeds 32768");
  std::vector<rw_surface> sf(surfaces, surfaces + n_surf);
  sf[s1].carries_doe = 0;
  rw_config c2 = *cfg;
  c2.rays_side = cfg->rays_side * n1;
  c2.n_ssr = n_ssr2;
  const CascSpec cs = {s1, *doe1, cfg->rays_side, n1,
                       cfg->sampling == RW_SAMPLE_FULL ? M * M : cfg->n_ssr};
  return plan_create(sf.data(), n_surf, doe2, params, n_params, &c2, &cs, out);
}

rw_status rw_plan_workspace_bytes(const rw_plan* pl, size_t* fwd_bytes, size_t* bwd_extra_bytes) {
  if (!pl || !fwd_bytes) return fail(RW_ERR_INVALID_ARG, "null argument");
  *fwd_bytes = pl->fwd_bytes;
  if (bwd_extra_bytes) *bwd_extra_bytes = pl->total - pl->fwd_bytes;
  return RW_OK;
}

rw_status rw_plan_destroy(rw_plan* pl) {
  if (!pl) return RW_OK;
  (void)hipFree(pl->d_cfg);
  (void)hipFree(pl->d_cfg1);
  (void)hipFree(pl->d_pairs);
  (void)hipFree(pl->d_base);
  (void)hipFree(pl->d_prm);
  for (int i = 0; i < 4; ++i) (void)hipFree(pl->d_tw_cls[i]);
  (void)hipFree(pl->d_tw_nf);
  (void)hipFree(pl->d_psi);
  for (auto& e : pl->ev_used) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
  for (auto& e : pl->ev_pool) (void)hipEventDestroy(e);
  pl->gfwd.reset();
  pl->gbwd.reset();
  pl->gstep.reset();
  if (pl->cap_st) (void)hipStreamDestroy(pl->cap_st);
  delete pl;
  return RW_OK;
}

rw_status rw_autotune(rw_plan* pl, void* ws, size_t ws_bytes, int* shape_out, void* stream) {
  if (!pl || !ws) return fail(RW_ERR_INVALID_ARG, "null argument");
  if (pl->casc) return fail(RW_ERR_UNSUPPORTED, "rw_autotune does not tune a DOE cascade");
  if (pl->cfg.deterministic)
    return fail(RW_ERR_UNSUPPORTED, "the deterministic mode is forward-only: nothing to tune");
  if (!pl->fwd_done || !pl->fwd_full || ws != pl->fwd_ws || ws_bytes < pl->total)
    return fail(RW_ERR_STATE, "rw_autotune needs a preceding rw_forward on this workspace "
                              "(of fwd + bwd bytes)");
  hipStream_t st = (hipStream_t)stream;
  char* b = (char*)ws;
  pl->gfwd.reset();
  pl->gbwd.reset();
  pl->gstep.reset();
  const bool prof = pl->prof;
  pl->prof = false;
  DoeArgs a = doe_args(pl, ws, pl->fwd_replay, nullptr);
  a.adj = b + pl->off_grid;
  a.interp = pl->tiled_interp ? (const void*)(b + pl->off_interp) : nullptr;
  a.g2 = pl->g2 ? (void*)(b + pl->off_g2) : nullptr;
  a.want_lens = 0;
  a.ray0 = 0;
  // tune on the first pairs only, about 2^19 rays (the launch shape does not
  // depend on which rays, only on how many per workgroup)
  const int ppg = std::max(1, std::min(pl->group_pairs, (int)(((size_t)1 << 19) / pl->R2)));
  a.nray = (size_t)ppg * pl->R2;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int blocks_c[4] = {256, 512, 1024, 2048};
  const int rb_c[3] = {4, 8, 16};
  rw_status res = RW_OK;
  for (int dir = 0; dir < 2 && res == RW_OK; ++dir) {
    const bool fwd = dir == 0;
    float best = 1e30f;
    int bb = pl->blocks_dir[dir], br = pl->rb_dir[dir];
    for (int i = 0; i < 4 && res == RW_OK; ++i) {
      if (blocks_c[i] > pl->doe_blocks) continue;
      for (int j = 0; j < 3 && res == RW_OK; ++j) {
        pl->blocks_dir[dir] = blocks_c[i];
        pl->rb_dir[dir] = rb_c[j];
        // one untimed launch, then one timed
        res = doe_launch(pl, fwd, a, 0, ppg, st);
        if (res != RW_OK) break;
        (void)hipEventRecord(e0, st);
        res = doe_launch(pl, fwd, a, 0, ppg, st);
        (void)hipEventRecord(e1, st);
        if (res != RW_OK) break;
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          res = fail(RW_ERR_HIP, "rw_autotune: event timing failed");
          break;
        }
        if (ms < best) { best = ms; bb = blocks_c[i]; br = rb_c[j]; }
      }
    }
    pl->blocks_dir[dir] = bb;
    pl->rb_dir[dir] = br;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  pl->prof = prof;
  pl->fwd_done = false;             // the trial launches overwrote forward state
  if (shape_out) {
    shape_out[0] = pl->blocks_dir[0]; shape_out[1] = pl->rb_dir[0];
    shape_out[2] = pl->blocks_dir[1]; shape_out[3] = pl->rb_dir[1];
  }
  return res;
}

rw_status rw_set_launch_shape(rw_plan* pl, const int* shape) {
  if (!pl || !shape) return fail(RW_ERR_INVALID_ARG, "null argument");
  for (int dir = 0; dir < 2; ++dir) {
    const int nb = shape[2 * dir], rb = shape[2 * dir + 1];
    if (nb < 1 || nb > pl->doe_blocks || (rb != 4 && rb != 8 && rb != 16))
      return fail(RW_ERR_INVALID_ARG, "launch shape: workgroups in [1, " +
                                          std::to_string(pl->doe_blocks) +
                                          "], ray block side 4, 8 or 16");
  }
  pl->blocks_dir[0] = shape[0]; pl->rb_dir[0] = shape[1];
  pl->blocks_dir[1] = shape[2]; pl->rb_dir[1] = shape[3];
  pl->gfwd.reset();
  pl->gbwd.reset();
  pl->gstep.reset();
  return RW_OK;
}

// Adam update, one thread per parameter; the bias corrections are formed on the
// host in double.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2, float lo, float hi) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  float q = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  if (lo <= hi) q = fminf(fmaxf(q, lo), hi);
  p[i] = q;
}

rw_status rw_adam_step(float* params, const float* grads, float* m, float* v, size_t n,
                       float lr, float beta1, float beta2, float eps, int t, float lo,
                       float hi, void* stream) {
  if (n == 0) return RW_OK;
  if (!params || !grads || !m || !v) return fail(RW_ERR_INVALID_ARG, "null array");
  if (t < 1 || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps > 0.0f))
    return fail(RW_ERR_INVALID_ARG, "bad Adam step number or hyper-parameters");
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, t)));
  const unsigned int blocks = (unsigned int)((n + 255) / 256);
  hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(256), 0, (hipStream_t)stream, params, grads, m,
                     v, n, lr, beta1, beta2, eps, c1, c2, lo, hi);
  HIPCHK(hipGetLastError());
  return RW_OK;
}

rw_status rw_patch_dft(int M, int P, long long n, const void* in, void* out, void* stream) {
  if (n < 0 || (n > 0 && (!in || !out))) return fail(RW_ERR_INVALID_ARG, "bad patch arrays");
  if (!(M == 16 || M == 32 || M == 64) || P < 1 || P > M)
    return fail(RW_ERR_SHAPE, "rw_patch_dft takes M in {16, 32, 64} and 1 <= P <= M");
  if (n == 0) return RW_OK;
  HIPCHK(launch_patch_dft(M, P, n, in, out, (hipStream_t)stream));
  return RW_OK;
}

rw_status rw_set_graph(rw_plan* pl, int enable) {
  if (!pl) return fail(RW_ERR_INVALID_ARG, "null plan");
  pl->graph = enable != 0;
  if (!pl->graph) {
    pl->gfwd.reset();
    pl->gbwd.reset();
    pl->gstep.reset();
  }
  return RW_OK;
}

// The launches of one forward pass, in stream order: the prologue (live
// prescription, transmission map, counters), each launch group of pairs, and the
// loss of Eq. 5.
static rw_status fwd_prologue(rw_plan* pl, const float* lens_params, const float* doe_phase,
                              const float* doe_amp, void* ws, hipStream_t st) {
  char* b = (char*)ws;
  const bool dbl_f = pl->cfg.precision == RW_PREC_FP64;
  pl->cur_phase = doe_phase;
  hipLaunchKernelGGL(k_params, dim3(1), dim3(1), 0, st, pl->d_cfg, pl->d_base, pl->base_sensor_z,
                     pl->d_prm, lens_params, (DevLive*)(b + pl->off_live));
  const int nmap = pl->H * pl->W;
  // a cascade's maps are [2][H][W]: the first DOE's, then the second's (the plan's)
  for (int k = 0; k < (pl->casc ? 2 : 1); ++k) {
    void* dst = b + (pl->casc && k == 0 ? pl->off_tmap1 : pl->off_tmap);
    const size_t o = pl->casc ? (size_t)k * nmap : 0;
    if (dbl_f)
      hipLaunchKernelGGL(k_tmap<double>, dim3((nmap + 255) / 256), dim3(256), 0, st, doe_phase + o,
                         doe_amp + o, (C2<double>*)dst, nmap, pl->doe.field);
    else
      hipLaunchKernelGGL(k_tmap<float>, dim3((nmap + 255) / 256), dim3(256), 0, st, doe_phase + o,
                         doe_amp + o, (C2<float>*)dst, nmap, pl->doe.field);
    HIPCHK(hipGetLastError());
  }
  zero<unsigned long long>(b + pl->off_stats, RW_N_STATS, st);
  return RW_OK;
}

// A launch group of a two-DOE cascade: launched rays to the first DOE, its
// patches, draws and relay of every secondary to the second DOE (the second
// DOE's incident rays), their patches and draws, then the records' Eq. 2 sum.
static rw_status fwd_group_cascade(rw_plan* pl, void* ws, const int32_t* replay_idx,
                                   int32_t* idx_out, float* psf_out, int pair0, int ppg,
                                   hipStream_t st) {
  char* b = (char*)ws;
  const DevLive* live = (const DevLive*)(b + pl->off_live);
  // the second DOE's sample indices follow the first DOE's
  const size_t off2 = pl->n1_total * (size_t)pl->N1;
  DoeArgs a1 = doe_args(pl, ws, replay_idx, idx_out);
  a1.cfg = pl->d_cfg1;
  a1.st = (const double*)(b + pl->off_st1);
  a1.n_total = pl->n1_total;
  a1.tmap = b + pl->off_tmap1;
  a1.ctx = (RayCtx*)(b + pl->off_ctx1);
  a1.ray_class = (unsigned char*)(b + pl->off_rcls1);
  a1.emit = pl->N1;
  a1.rec_pos = nullptr;
  a1.rec_val = nullptr;
  a1.jdraw = pl->fwd_only || pl->cfg.sampling == RW_SAMPLE_FULL ? nullptr
                                                                : (int32_t*)(b + pl->off_jdraw1);
  a1.relay = (double*)(b + pl->off_st);
  a1.relay_n = pl->n_total;
  a1.cfg2 = pl->d_cfg;
  const size_t nr1 = (size_t)ppg * pl->R1sq;
  a1.ray0 = (size_t)pair0 * pl->R1sq;
  a1.nray = nr1;
  const int tb1 = (int)((nr1 + 255) / 256);
  {
    StageTimer tm_(pl, RW_STAGE_TRACE, st);
    if (pl->cfg.precision == RW_PREC_FP32)
      hipLaunchKernelGGL(k_trace<float>, dim3(tb1), dim3(256), 0, st, pl->d_cfg1, pl->d_pairs,
                         live, (double*)(b + pl->off_st1), (double*)(b + pl->off_ck1),
                         pl->n1_total, pair0, ppg, (unsigned long long*)(b + pl->off_stats));
    else
      hipLaunchKernelGGL(k_trace<double>, dim3(tb1), dim3(256), 0, st, pl->d_cfg1, pl->d_pairs,
                         live, (double*)(b + pl->off_st1), (double*)(b + pl->off_ck1),
                         pl->n1_total, pair0, ppg, (unsigned long long*)(b + pl->off_stats));
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_ray_ctx, dim3(tb1), dim3(256), 0, st, a1);
    HIPCHK(hipGetLastError());
  }
  rw_status s;
  {
    StageTimer tm_(pl, RW_STAGE_DOE_FWD, st);
    s = doe_launch(pl, true, a1, pair0, ppg, st, pl->R1);
  }
  if (s != RW_OK) return s;
  DoeArgs a2 = doe_args(pl, ws, replay_idx ? replay_idx + off2 : nullptr,
                        idx_out ? idx_out + off2 : nullptr);
  a2.ain = (const double*)(b + pl->off_st) + 8 * pl->n_total;
  const size_t nr2 = (size_t)ppg * pl->R2;
  a2.ray0 = (size_t)pair0 * pl->R2;
  a2.nray = nr2;
  {
    StageTimer tm_(pl, RW_STAGE_TRACE, st);
    hipLaunchKernelGGL(k_ray_ctx, dim3((int)((nr2 + 255) / 256)), dim3(256), 0, st, a2);
    HIPCHK(hipGetLastError());
  }
  {
    StageTimer tm_(pl, RW_STAGE_DOE_FWD, st);
    s = doe_launch(pl, true, a2, pair0, ppg, st);
  }
  if (s != RW_OK) return s;
  s = bin_and_spread(pl, ws, st, pair0, ppg);
  if (s != RW_OK) return s;
  StageTimer tm_(pl, RW_STAGE_GRID_FWD, st);
  return grid_fwd(pl, ws, st, pair0, ppg, psf_out);
}

static rw_status fwd_group(rw_plan* pl, void* ws, const int32_t* replay_idx, int32_t* idx_out,
                           float* psf_out, int pair0, int ppg, hipStream_t st) {
  if (pl->casc) return fwd_group_cascade(pl, ws, replay_idx, idx_out, psf_out, pair0, ppg, st);
  char* b = (char*)ws;
  DoeArgs a = doe_args(pl, ws, replay_idx, idx_out);
  const size_t nr = (size_t)ppg * pl->R2;
  const int tb = (int)((nr + 255) / 256);
  {
    StageTimer tm_(pl, RW_STAGE_TRACE, st);
    if (pl->cfg.precision == RW_PREC_FP32)
      hipLaunchKernelGGL(k_trace<float>, dim3(tb), dim3(256), 0, st, pl->d_cfg, pl->d_pairs,
                         (const DevLive*)(b + pl->off_live), (double*)(b + pl->off_st),
                         (double*)(b + pl->off_ck), pl->n_total, pair0, ppg,
                         (unsigned long long*)(b + pl->off_stats));
    else
      hipLaunchKernelGGL(k_trace<double>, dim3(tb), dim3(256), 0, st, pl->d_cfg, pl->d_pairs,
                         (const DevLive*)(b + pl->off_live), (double*)(b + pl->off_st),
                         (double*)(b + pl->off_ck), pl->n_total, pair0, ppg,
                         (unsigned long long*)(b + pl->off_stats));
  }
  HIPCHK(hipGetLastError());
  a.ray0 = (size_t)pair0 * pl->R2;
  a.nray = nr;
  {
    StageTimer tm_(pl, RW_STAGE_TRACE, st);
    hipLaunchKernelGGL(k_ray_ctx, dim3(tb), dim3(256), 0, st, a);
  }
  HIPCHK(hipGetLastError());
  rw_status s;
  {
    StageTimer tm_(pl, RW_STAGE_DOE_FWD, st);
    s = doe_launch(pl, true, a, pair0, ppg, st);
  }
  if (s != RW_OK) return s;
  s = bin_and_spread(pl, ws, st, pair0, ppg);
  if (s != RW_OK) return s;
  StageTimer tm_(pl, RW_STAGE_GRID_FWD, st);
  return grid_fwd(pl, ws, st, pair0, ppg, psf_out);
}

static void loss_pairs(rw_plan* pl, void* ws, const float* psf_out, const float* target,
                       int pair0, int ppg, hipStream_t st) {
  char* b = (char*)ws;
  hipLaunchKernelGGL(k_loss_pairs, dim3(ppg), dim3(256), 0, st, psf_out, target, pl->Q * pl->Q,
                     pair0, (double*)(b + pl->off_alpha), (double*)(b + pl->off_lossp));
}

static void loss_total(rw_plan* pl, void* ws, float* loss_out, hipStream_t st) {
  char* b = (char*)ws;
  hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(64), 0, st, (const double*)(b + pl->off_lossp),
                     pl->n_pairs, loss_out);
}

static rw_status fwd_enqueue(rw_plan* pl, const float* lens_params, const float* doe_phase,
                             const float* doe_amp, const float* target, float* psf_out,
                             float* loss_out, void* ws, const int32_t* replay_idx,
                             int32_t* idx_out, hipStream_t st) {
  rw_status s = fwd_prologue(pl, lens_params, doe_phase, doe_amp, ws, st);
  if (s != RW_OK) return s;
  for (int pair0 = 0; pair0 < pl->n_pairs; pair0 += pl->group_pairs) {
    const int ppg = std::min(pl->group_pairs, pl->n_pairs - pair0);
    s = fwd_group(pl, ws, replay_idx, idx_out, psf_out, pair0, ppg, st);
    if (s != RW_OK) return s;
  }
  if (target) {
    loss_pairs(pl, ws, psf_out, target, 0, pl->n_pairs, st);
    loss_total(pl, ws, loss_out, st);
    HIPCHK(hipGetLastError());
  }
  return RW_OK;
}

static rw_status forward_impl(rw_plan* pl, const float* lens_params, const float* doe_phase,
                              const float* doe_amp, const float* target, float* psf_out,
                              float* loss_out, void* ws, bool fwd_only, bool use_graph,
                              const int32_t* replay_idx, int32_t* idx_out, hipStream_t st) {
  pl->fwd_done = false;
  pl->fwd_only = fwd_only;
  rw_status r;
  if (use_graph) {
    const GraphKey key = {{(const void*)lens_params, doe_phase, doe_amp, target, psf_out, loss_out,
                           ws, replay_idx, idx_out, fwd_only ? (const void*)1 : nullptr}};
    r = graph_run(pl, pl->gfwd, key, st, [&](hipStream_t cs) {
      return fwd_enqueue(pl, lens_params, doe_phase, doe_amp, target, psf_out, loss_out, ws,
                         replay_idx, idx_out, cs);
    });
  } else {
    r = fwd_enqueue(pl, lens_params, doe_phase, doe_amp, target, psf_out, loss_out, ws,
                    replay_idx, idx_out, st);
  }
  pl->fwd_only = false;
  if (r != RW_OK) return r;
  pl->fwd_done = true;
  pl->fwd_full = !fwd_only;
  pl->fwd_target = target;
  pl->fwd_replay = replay_idx;
  pl->fwd_phase = doe_phase;
  pl->fwd_psf = psf_out;
  pl->fwd_amp = doe_amp;
  pl->fwd_ws = ws;
  pl->fwd_stream = st;
  return RW_OK;
}

static rw_status forward_args(const rw_plan* pl, const float* lens_params, const float* doe_phase,
                              const float* doe_amp, const float* target, const float* psf_out,
                              const float* loss_out, const int32_t* replay_idx) {
  if (!pl || !doe_phase || !doe_amp || !psf_out)
    return fail(RW_ERR_INVALID_ARG, "null required argument");
  if (pl->prm.size() > 0 && !lens_params)
    return fail(RW_ERR_INVALID_ARG, "lens_params required when the plan has lens parameters");
  if (target && !loss_out) return fail(RW_ERR_INVALID_ARG, "target given without loss_out");
  if (replay_idx && pl->cfg.sampling == RW_SAMPLE_FULL)
    return fail(RW_ERR_INVALID_ARG, "replay is meaningless in FULL sampling");
  return RW_OK;
}

rw_status rw_forward(rw_plan* pl, const float* lens_params, const float* doe_phase,
                     const float* doe_amp, const float* target, float* psf_out, float* loss_out,
                     void* ws, size_t ws_bytes, const int32_t* replay_idx, int32_t* idx_out,
                     void* stream) {
  const rw_status a = forward_args(pl, lens_params, doe_phase, doe_amp, target, psf_out, loss_out,
                                   replay_idx);
  if (a != RW_OK) return a;
  if (!ws) return fail(RW_ERR_INVALID_ARG, "null workspace");
  if (ws_bytes < pl->fwd_bytes)
    return fail(RW_ERR_STATE, "workspace smaller than the forward bytes of rw_plan_workspace_bytes");
  if (((uintptr_t)ws & 255) != 0) return fail(RW_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (pl->cfg.check_finite) {
    hipStream_t st = (hipStream_t)stream;
    unsigned int* flag = (unsigned int*)((char*)ws + pl->off_stats);
    zero<unsigned int>(flag, 1, st);
    const size_t nmap = (size_t)pl->H * pl->W * (pl->casc ? 2 : 1);
    const size_t nt = target ? (size_t)pl->n_pairs * pl->Q * pl->Q : 0;
    hipLaunchKernelGGL(k_check_finite, dim3(1024), dim3(256), 0, st, lens_params,
                       lens_params ? pl->prm.size() : (size_t)0, doe_phase, nmap, doe_amp, nmap,
                       target, nt, flag);
    HIPCHK(hipGetLastError());
    unsigned int h = 0;
    HIPCHK(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h) {
      pl->fwd_done = false;
      return fail(RW_ERR_NONFINITE, "NaN or Inf in lens_params, doe_phase, doe_amp or target");
    }
  }
  return forward_impl(pl, lens_params, doe_phase, doe_amp, target, psf_out, loss_out, ws,
                      ws_bytes < pl->total, pl->graph, replay_idx, idx_out, (hipStream_t)stream);
}

}  // extern "C"

// ------------------------------------------------- forward without allocation ---
// The device workspace of rw_forward_static: one array per GPU the library runs
// on, held until the process ends.  Host code never uses the array's name as an
// address; it takes the device address from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[RW_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once per device,
// with the device current).
rw_status static_scratch(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(RW_ERR_UNSUPPORTED, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(RW_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RW_OK;
}
}  // namespace

extern "C" {

rw_status rw_forward_static(rw_plan* pl, const float* lens_params, const float* doe_phase,
                            const float* doe_amp, const float* target, float* psf_out,
                            float* loss_out, const int32_t* replay_idx, int32_t* idx_out,
                            void* stream) {
  const rw_status a = forward_args(pl, lens_params, doe_phase, doe_amp, target, psf_out, loss_out,
                                   replay_idx);
  if (a != RW_OK) return a;
  if (pl->fwd_bytes > RW_STATIC_SCRATCH_BYTES)
    return fail(RW_ERR_UNSUPPORTED,
                "the plan's forward workspace (" + std::to_string(pl->fwd_bytes) +
                    " bytes) exceeds the static scratch of rw_forward_static (" +
                    std::to_string(RW_STATIC_SCRATCH_BYTES) + " bytes)");
  void* ws = nullptr;
  const rw_status e = static_scratch(&ws);
  if (e != RW_OK) return e;
  pl->no_alloc = true;
  const rw_status r = forward_impl(pl, lens_params, doe_phase, doe_amp, target, psf_out, loss_out,
                                   ws, true, false, replay_idx, idx_out, (hipStream_t)stream);
  pl->no_alloc = false;
  return r;
}

rw_status rw_set_profiling(rw_plan* pl, int enable) {
  if (!pl) return fail(RW_ERR_INVALID_ARG, "null plan");
  for (auto& e : pl->ev_used) { pl->ev_pool.push_back(e.a); pl->ev_pool.push_back(e.b); }
  pl->ev_used.clear();
  pl->prof = enable != 0;
  return RW_OK;
}

rw_status rw_get_profile(rw_plan* pl, rw_profile* out) {
  if (!pl || !out) return fail(RW_ERR_INVALID_ARG, "null argument");
  memset(out, 0, sizeof(*out));
  for (auto& e : pl->ev_used) {
    HIPCHK(hipEventSynchronize(e.b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e.a, e.b));
    out->ms[e.stage] += ms;
    out->launches[e.stage] += 1;
  }
  return RW_OK;
}

rw_status rw_get_stats(rw_plan* pl, rw_stats* out) {
  if (!pl || !out) return fail(RW_ERR_INVALID_ARG, "null argument");
  if (!pl->fwd_done) return fail(RW_ERR_STATE, "no forward pass yet");
  unsigned long long h[RW_N_STATS];
  HIPCHK(hipStreamSynchronize(pl->fwd_stream));
  HIPCHK(hipMemcpy(h, (char*)pl->fwd_ws + pl->off_stats, sizeof(h), hipMemcpyDeviceToHost));
  out->rays_total = pl->n_total;
  out->rays_alive = h[RW_ST_ALIVE];
  out->secondaries = h[RW_ST_SEC];
  out->killed_no_hit = h[RW_ST_NOHIT];
  out->killed_aperture = h[RW_ST_APER];
  out->killed_tir = h[RW_ST_TIR];
  out->killed_outside_doe = h[RW_ST_OUTSIDE];
  out->secondaries_lost = h[RW_ST_LOST];
  out->evanescent_bins = h[RW_ST_EVAN];
  out->spectrum_bins = h[RW_ST_BINS];
  for (int c = 0; c < 4; ++c) out->rays_by_class[c] = h[RW_ST_CLASS0 + c];
  return RW_OK;
}

rw_status rw_export_doe_hits(const rw_plan* pl, const void* ws, double* out, void* stream) {
  if (!pl || !ws || !out) return fail(RW_ERR_INVALID_ARG, "null argument");
  hipStream_t st = (hipStream_t)stream;
  const size_t n = pl->n_total;
  hipLaunchKernelGGL(k_export_state, dim3((unsigned)((8 * n + 255) / 256)), dim3(256), 0, st,
                     (const double*)((const char*)ws + pl->off_st), n, out);
  HIPCHK(hipGetLastError());
  return RW_OK;
}

// The launches of one backward pass, in stream order: clearing the gradient
// accumulators, each launch group of pairs, and the final maps.
static void bwd_prologue(rw_plan* pl, void* ws, bool want_lens, hipStream_t st) {
  char* b = (char*)ws;
  const bool dbl = pl->cfg.precision == RW_PREC_FP64;
  const size_t nmap = (size_t)pl->H * pl->W;
  if (dbl) zero<double>(b + pl->off_gt, 2 * nmap, st);
  else zero<float>(b + pl->off_gt, 2 * nmap, st);
  zero<double>(b + pl->off_lensg, RW_LENSG_SLOTS, st);
  if (want_lens) zero<double>(b + pl->off_raygrad, (size_t)RW_RAYGRAD * pl->n_total, st);
  const size_t nacc = (size_t)pl->blocks_dir[1] * pl->acc_side * pl->acc_side * 2;
  if (dbl) zero<double>(b + pl->off_acc, nacc, st);
  else zero<float>(b + pl->off_acc, nacc, st);
}

// tiled: the group's binned records of the forward are still in the workspace
static rw_status bwd_group(rw_plan* pl, const float* dL_dpsf, void* ws, bool want_lens,
                           bool tiled, int pair0, int ppg, hipStream_t st) {
  char* b = (char*)ws;
  DoeArgs a = doe_args(pl, ws, pl->fwd_replay, nullptr);
  a.adj = b + pl->off_grid;
  a.interp = tiled ? (const void*)(b + pl->off_interp) : nullptr;
  a.g2 = pl->g2 ? (void*)(b + pl->off_g2) : nullptr;
  a.want_lens = want_lens ? 1 : 0;
  a.stats = nullptr;
  if (pl->casc) {
    // the second DOE of a cascade: records carry the incident amplitude
    a.ain = (const double*)(b + pl->off_st) + 8 * pl->n_total;
    a.gain = (double*)(b + pl->off_gain);
  }
  rw_status s;
  {
    StageTimer tm_(pl, RW_STAGE_GRID_BWD, st);
    s = grid_bwd(pl, ws, st, pair0, ppg, dL_dpsf);
  }
  if (s != RW_OK) return s;
  if (tiled) {
    s = interp_tiles(pl, ws, st, pair0, ppg);
    if (s != RW_OK) return s;
  }
  const size_t nr = (size_t)ppg * pl->R2;
  a.ray0 = (size_t)pair0 * pl->R2;
  a.nray = nr;
  {
    StageTimer tm_(pl, RW_STAGE_DOE_BWD, st);
    s = doe_launch(pl, false, a, pair0, ppg, st);
  }
  if (s != RW_OK) return s;
  if (want_lens && pl->has_post) {
    StageTimer tm_(pl, RW_STAGE_TRACE_BWD, st);
    const unsigned nb = (unsigned)((nr + 3) / 4);
    if (pl->cfg.precision == RW_PREC_FP64)
      hipLaunchKernelGGL(k_post_bwd<double>, dim3(nb), dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL(k_post_bwd<float>, dim3(nb), dim3(256), 0, st, a);
    HIPCHK(hipGetLastError());
  }
  if (want_lens) {
    StageTimer tm_(pl, RW_STAGE_TRACE_BWD, st);
    hipLaunchKernelGGL(k_trace_bwd, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st,
                       pl->d_cfg, pl->d_pairs, (const DevLive*)(b + pl->off_live),
                       (const double*)(b + pl->off_st), (const double*)(b + pl->off_ck),
                       (const double*)(b + pl->off_raygrad), pl->n_total, a.ray0, nr,
                       (double*)(b + pl->off_lensg));
    HIPCHK(hipGetLastError());
  }
  return RW_OK;
}

static rw_status bwd_epilogue(rw_plan* pl, void* ws, float* d_phase, float* d_amp, float* d_lens,
                              bool want_lens, hipStream_t st) {
  char* b = (char*)ws;
  const int n = pl->H * pl->W;
  if (pl->cfg.precision == RW_PREC_FP64)
    hipLaunchKernelGGL(k_dmaps<double>, dim3((n + 255) / 256), dim3(256), 0, st,
                       (const float*)pl->fwd_phase, (const float*)pl->fwd_amp,
                       (const C2<double>*)(b + pl->off_gt), d_phase, d_amp, n, pl->doe.field);
  else
    hipLaunchKernelGGL(k_dmaps<float>, dim3((n + 255) / 256), dim3(256), 0, st,
                       (const float*)pl->fwd_phase, (const float*)pl->fwd_amp,
                       (const C2<float>*)(b + pl->off_gt), d_phase, d_amp, n, pl->doe.field);
  if (want_lens)
    hipLaunchKernelGGL(k_lens_map, dim3(1), dim3(64), 0, st, pl->d_cfg, pl->d_prm,
                       (const double*)(b + pl->off_lensg), d_lens);
  HIPCHK(hipGetLastError());
  return RW_OK;
}

// Backward of a two-DOE cascade (map gradients; the relayed rays' geometry
// follows from the drawn bins, so the maps act through the amplitudes alone):
// the second DOE's adjoint, which also leaves dL/d(incident amplitude) per ray,
// then the first DOE's, whose draws take those as their weight cogradients.
static rw_status bwd_enqueue_cascade(rw_plan* pl, const float* dL_dpsf, float* d_phase,
                                     float* d_amp, void* ws, hipStream_t st) {
  char* b = (char*)ws;
  bwd_prologue(pl, ws, false, st);
  const size_t nmap = (size_t)pl->H * pl->W;
  if (pl->cfg.precision == RW_PREC_FP64) zero<double>(b + pl->off_gt1, 2 * nmap, st);
  else zero<float>(b + pl->off_gt1, 2 * nmap, st);
  zero<double>(b + pl->off_gain, 2 * pl->n_total, st);
  for (int pair0 = 0; pair0 < pl->n_pairs; pair0 += pl->group_pairs) {
    const int ppg = std::min(pl->group_pairs, pl->n_pairs - pair0);
    const rw_status s = bwd_group(pl, dL_dpsf, ws, false, pl->tiled_interp, pair0, ppg, st);
    if (s != RW_OK) return s;
  }
  for (int pair0 = 0; pair0 < pl->n_pairs; pair0 += pl->group_pairs) {
    const int ppg = std::min(pl->group_pairs, pl->n_pairs - pair0);
    DoeArgs a1 = doe_args(pl, ws, nullptr, nullptr);
    a1.cfg = pl->d_cfg1;
    a1.st = (const double*)(b + pl->off_st1);
    a1.n_total = pl->n1_total;
    a1.tmap = b + pl->off_tmap1;
    a1.ctx = (RayCtx*)(b + pl->off_ctx1);
    a1.ray_class = (unsigned char*)(b + pl->off_rcls1);
    a1.emit = pl->N1;
    a1.rec_pos = nullptr;
    a1.rec_val = nullptr;
    a1.jdraw = pl->cfg.sampling == RW_SAMPLE_FULL ? nullptr : (int32_t*)(b + pl->off_jdraw1);
    a1.gt = b + pl->off_gt1;
    a1.relay = (double*)(b + pl->off_st);
    a1.relay_n = pl->n_total;
    a1.cfg2 = pl->d_cfg;
    a1.gain = (double*)(b + pl->off_gain);
    a1.want_lens = 0;
    a1.stats = nullptr;
    a1.ray0 = (size_t)pair0 * pl->R1sq;
    a1.nray = (size_t)ppg * pl->R1sq;
    StageTimer tm_(pl, RW_STAGE_DOE_BWD, st);
    const rw_status s = doe_launch(pl, false, a1, pair0, ppg, st, pl->R1);
    if (s != RW_OK) return s;
  }
  // maps: the first DOE's dL/dt, then the second's
  const int n = (int)nmap;
  for (int k = 0; k < 2; ++k) {
    const size_t o = (size_t)k * nmap;
    void* g = b + (k == 0 ? pl->off_gt1 : pl->off_gt);
    if (pl->cfg.precision == RW_PREC_FP64)
      hipLaunchKernelGGL(k_dmaps<double>, dim3((n + 255) / 256), dim3(256), 0, st,
                         pl->fwd_phase + o, pl->fwd_amp + o, (const C2<double>*)g, d_phase + o,
                         d_amp + o, n, pl->doe.field);
    else
      hipLaunchKernelGGL(k_dmaps<float>, dim3((n + 255) / 256), dim3(256), 0, st,
                         pl->fwd_phase + o, pl->fwd_amp + o, (const C2<float>*)g, d_phase + o,
                         d_amp + o, n, pl->doe.field);
  }
  HIPCHK(hipGetLastError());
  return RW_OK;
}

static rw_status bwd_enqueue(rw_plan* pl, const float* dL_dpsf, float* d_phase, float* d_amp,
                             float* d_lens, void* ws, bool want_lens, hipStream_t st) {
  if (pl->casc) return bwd_enqueue_cascade(pl, dL_dpsf, d_phase, d_amp, ws, st);
  bwd_prologue(pl, ws, want_lens, st);
  for (int pair0 = 0; pair0 < pl->n_pairs; pair0 += pl->group_pairs) {
    const int ppg = std::min(pl->group_pairs, pl->n_pairs - pair0);
    const rw_status s = bwd_group(pl, dL_dpsf, ws, want_lens, pl->tiled_interp, pair0, ppg, st);
    if (s != RW_OK) return s;
  }
  return bwd_epilogue(pl, ws, d_phase, d_amp, d_lens, want_lens, st);
}

// One training step on the loss of Eq. 5: the pairs' losses and cogradients are
// independent, so each launch group runs its backward right after its forward,
// while its binned records are still in the workspace (tiled interpolation in
// every group), then the maps and the loss are finished.
static rw_status step_enqueue(rw_plan* pl, const float* lens_params, const float* doe_phase,
                              const float* doe_amp, const float* target, float* psf_out,
                              float* loss_out, float* d_phase, float* d_amp, float* d_lens,
                              void* ws, bool want_lens, hipStream_t st) {
  rw_status s = fwd_prologue(pl, lens_params, doe_phase, doe_amp, ws, st);
  if (s != RW_OK) return s;
  bwd_prologue(pl, ws, want_lens, st);
  const bool tiled = pl->tiled_interp || pl->tiled_groups;
  for (int pair0 = 0; pair0 < pl->n_pairs; pair0 += pl->group_pairs) {
    const int ppg = std::min(pl->group_pairs, pl->n_pairs - pair0);
    s = fwd_group(pl, ws, nullptr, nullptr, psf_out, pair0, ppg, st);
    if (s != RW_OK) return s;
    loss_pairs(pl, ws, psf_out, target, pair0, ppg, st);
    s = bwd_group(pl, nullptr, ws, want_lens, tiled, pair0, ppg, st);
    if (s != RW_OK) return s;
  }
  loss_total(pl, ws, loss_out, st);
  return bwd_epilogue(pl, ws, d_phase, d_amp, d_lens, want_lens, st);
}

rw_status rw_backward(rw_plan* pl, const float* dL_dpsf, float* d_phase, float* d_amp,
                      float* d_lens, void* ws, size_t ws_bytes, void* stream) {
  if (!pl || !d_phase || !d_amp || !ws) return fail(RW_ERR_INVALID_ARG, "null required argument");
  if (pl->cfg.deterministic)
    return fail(RW_ERR_UNSUPPORTED, "the deterministic mode is forward-only (its gradient sums "
                                    "are not ordered)");
  if (pl->casc && d_lens && !pl->prm.empty())
    return fail(RW_ERR_UNSUPPORTED, "lens gradients through a DOE cascade are not built");
  if (!pl->fwd_done) return fail(RW_ERR_STATE, "rw_backward needs a preceding rw_forward");
  if (ws != pl->fwd_ws || ws_bytes < pl->total)
    return fail(RW_ERR_STATE, "rw_backward must use the workspace of the forward");
  if (!pl->fwd_full)
    return fail(RW_ERR_STATE, "the forward ran forward-only (its workspace held fwd bytes only)");
  if (!dL_dpsf && !pl->fwd_target)
    return fail(RW_ERR_STATE, "dL_dpsf is NULL and the forward had no target");
  const bool want_lens = pl->prm.size() > 0 && d_lens != nullptr;
  if (want_lens && pl->has_post && (!pl->tiled_interp || pl->n_surf - pl->s_doe - 1 > kPostMax))
    return fail(RW_ERR_UNSUPPORTED,
                "lens-parameter gradients through surfaces after the DOE need a batched plan "
                "whose records fit one launch group, and at most 4 such surfaces");
  hipStream_t st = (hipStream_t)stream;
  if (pl->graph) {
    // every pointer the recorded kernels read: the forward's PSF feeds the Eq. 5
    // cogradient when dL_dpsf is NULL
    const GraphKey key = {{(const void*)dL_dpsf, d_phase, d_amp, d_lens, ws, pl->fwd_replay,
                           pl->fwd_target, pl->fwd_phase, pl->fwd_amp, pl->fwd_psf}};
    return graph_run(pl, pl->gbwd, key, st, [&](hipStream_t cs) {
      return bwd_enqueue(pl, dL_dpsf, d_phase, d_amp, d_lens, ws, want_lens, cs);
    });
  }
  return bwd_enqueue(pl, dL_dpsf, d_phase, d_amp, d_lens, ws, want_lens, st);
}

rw_status rw_forward_backward(rw_plan* pl, const float* lens_params, const float* doe_phase,
                              const float* doe_amp, const float* target, float* psf_out,
                              float* loss_out, float* d_phase, float* d_amp, float* d_lens,
                              void* ws, size_t ws_bytes, void* stream) {
  if (pl && pl->casc)
    return fail(RW_ERR_UNSUPPORTED, "gradients through a DOE cascade are not built");
  if (pl && pl->cfg.deterministic)
    return fail(RW_ERR_UNSUPPORTED, "the deterministic mode is forward-only (its gradient sums "
                                    "are not ordered)");
  const rw_status a = forward_args(pl, lens_params, doe_phase, doe_amp, target, psf_out, loss_out,
                                   nullptr);
  if (a != RW_OK) return a;
  if (!target || !loss_out || !d_phase || !d_amp || !ws)
    return fail(RW_ERR_INVALID_ARG, "null required argument (target, loss_out, d_phase, d_amp, "
                                    "workspace)");
  if (ws_bytes < pl->total) return fail(RW_ERR_STATE, "workspace smaller than fwd + bwd bytes");
  if (((uintptr_t)ws & 255) != 0) return fail(RW_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  const bool want_lens = pl->prm.size() > 0 && d_lens != nullptr;
  const bool tiled = pl->tiled_interp || pl->tiled_groups;
  if (want_lens && pl->has_post && (!tiled || pl->n_surf - pl->s_doe - 1 > kPostMax))
    return fail(RW_ERR_UNSUPPORTED,
                "lens-parameter gradients through surfaces after the DOE need a batched plan "
                "and at most 4 such surfaces");
  hipStream_t st = (hipStream_t)stream;
  pl->fwd_done = false;
  pl->fwd_only = false;
  // the backward half reads the forward's state of this call
  pl->fwd_target = target;
  pl->fwd_replay = nullptr;
  pl->fwd_phase = doe_phase;
  pl->fwd_psf = psf_out;
  pl->fwd_amp = doe_amp;
  rw_status r;
  if (pl->graph) {
    const GraphKey key = {{(const void*)lens_params, doe_phase, doe_amp, target, psf_out, loss_out,
                           d_phase, d_amp, d_lens, ws}};
    r = graph_run(pl, pl->gstep, key, st, [&](hipStream_t cs) {
      return step_enqueue(pl, lens_params, doe_phase, doe_amp, target, psf_out, loss_out, d_phase,
                          d_amp, d_lens, ws, want_lens, cs);
    });
  } else {
    r = step_enqueue(pl, lens_params, doe_phase, doe_amp, target, psf_out, loss_out, d_phase,
                     d_amp, d_lens, ws, want_lens, st);
  }
  if (r != RW_OK) return r;
  // the draws and every pair's ray state are the forward's: a later rw_backward
  // recomputes what it needs (records of earlier groups are gone)
  pl->fwd_done = true;
  pl->fwd_full = true;
  pl->fwd_ws = ws;
  pl->fwd_stream = st;
  return RW_OK;
}

}  // extern "C"

