// C-ABI entry points of libmdpl (declared in include/mdpl.h).
//
// The host side validates arguments, carves the caller's workspace and
// enqueues kernels on the context's stream.  It owns no device memory.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "internal.h"
#include "mlp_args.h"

using namespace mdpl;

namespace {

int32_t g_last_hip_error = 0;

#define HIP_TRY(expr)                           \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) {                     \
      g_last_hip_error = (int32_t)e_;           \
      return MDPL_EHIP;                         \
    }                                           \
  } while (0)

struct Timing {
  std::vector<hipEvent_t> ev[2];  // start/stop pairs, flattened
  std::vector<hipEvent_t> pool;   // created, not recorded (reused across timed runs)
  int64_t launches[2] = {0, 0};   // launches of each kind since the last read
  int every = 1;                  // time launches 0, every, 2 every, ... of each kind
};

// run kinds whose state a continued run may take over
constexpr int kKindLJ = 1, kKindMLP = 2;

// The rule's host decision (see run_loop): records older than kLagMax steps
// make the host wait (without draining the stream) until the device is
// within kLagKeep steps; the prediction allows the largest speed of the
// recent records to double before the next record is seen.
constexpr int64_t kLagMax = 48, kLagKeep = 16;
constexpr double kSpeedHeadroom = 2.0;

}  // namespace

struct mdpl_sim {
  mdpl_lj_params p;
  hipStream_t st;
  Grid g;
  int64_t n, npad;
  double r2ext;
  LJConst c;
  int fbytes;
  SortBufs sort;
  int32_t* cell_start;
  int32_t* perm;         // sorted slot -> caller index of the last standalone build
  int32_t* skeys;        // sorted keys (points into sort buffers)
  TileList tl;
  double *sx, *sy, *sz;  // sorted positions (standalone) / alternate state (run)
  double *avx, *avy, *avz;
  void *afx, *afy, *afz;
  int32_t* aids;
  double *xb, *yb, *zb;  // positions at the last build (run)
  double *px, *py, *pz;  // spare positions: target of the fused drift (run)
  int32_t* offsets;      // n + 1 (export)
  double* partials;      // per-block partials
  int nblk;
  uint32_t* flags;
  int32_t* maxcount;
  double* max_disp;
  double* pe_w_tmp;      // 2 doubles
  bool built;
  bool have_list;
  bool timing;
  Timing tm;
  // run continuation: the arrays and kind of the last run (valid until an
  // mdpl_build or a failed run)
  struct {
    bool valid;
    int kind;
    StateArrays arrays;
  } resume;
  int64_t gstep;           // global step index of the current positions
  int64_t kb;              // gstep of the last list build of a run
  int64_t since;           // steps since that build
  bool have_ref;           // xb holds the positions of that build
  double* last_row;        // device: thermo row of the last step of the last run
  bool last_row_valid;
  // rebuild rule of Eq. extended_cutoff
  double* vpart[2];        // per-workgroup largest |v|^2 of the last two drifting launches
  int nvpart;              // capacity of each
  double* bound;
  KickRecord* ring_host;   // pinned, host-mapped
  KickRecord* ring_dev;
  KickTrack track;         // for the next drifting launch
  int pend_n;              // workgroups of the last drifting launch, its record not yet published (0: none)
  int64_t pend_step;       // the step index of that record
  int track_cur;           // slot of the next drifting launch's maxima
  int64_t n_rebuilds, n_early, n_syncs;
};

extern "C" {

const char* mdpl_status_string(mdpl_status s) {
  switch (s) {
    case MDPL_OK: return "ok";
    case MDPL_EINVAL: return "invalid argument";
    case MDPL_EBOX: return "box too small for the cell grid (need 3 cells of side >= rc+skin per axis)";
    case MDPL_ECAPACITY: return "neighbour-list capacity exceeded";
    case MDPL_ESKIN: return "particles moved half the skin before a list rebuild";
    case MDPL_ENONFINITE: return "non-finite velocity";
    case MDPL_EHIP: return "HIP runtime error";
    case MDPL_ESTATE: return "call out of order";
    case MDPL_EWORKSPACE: return "workspace too small or misaligned";
    case MDPL_ESCRATCH: return "input too large for the library's static scratch (MDPL_SCRATCH_BYTES)";
    default: return "unknown status";
  }
}

int32_t mdpl_last_hip_error(void) { return g_last_hip_error; }

}  // extern "C"

namespace {

mdpl_status validate(const mdpl_lj_params* p) {
  if (!p) return MDPL_EINVAL;
  if (p->n <= 0 || p->n > (1ll << 26)) return MDPL_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (!(p->box[k] > 0.0) || !isfinite(p->box[k])) return MDPL_EINVAL;
  if (!(p->rc > 0.0) || !(p->skin >= 0.0) || !(p->eps > 0.0) || !(p->sigma > 0.0) ||
      !(p->mass > 0.0) || !(p->dt > 0.0))
    return MDPL_EINVAL;
  if (!isfinite(p->rc) || !isfinite(p->skin) || !isfinite(p->dt)) return MDPL_EINVAL;
  if (p->reuse_every < 1 || p->reuse_every > kMaxCycle) return MDPL_EINVAL;
  if (p->shift < 0 || p->shift > 2) return MDPL_EINVAL;
  if (p->precision != MDPL_FP64 && p->precision != MDPL_FP32) return MDPL_EINVAL;
  if (p->max_nb < 1 || p->max_nb > 1024) return MDPL_EINVAL;
  if (p->pairs != MDPL_PAIRS_FULL && p->pairs != MDPL_PAIRS_HALF && p->pairs != MDPL_PAIRS_CELLS)
    return MDPL_EINVAL;
  if (p->rebuild != MDPL_REBUILD_FIXED && p->rebuild != MDPL_REBUILD_VMAX) return MDPL_EINVAL;
  Grid g;
  int unit[3] = {1, 1, 1};
  return make_grid(p->box, p->rc + p->skin, unit, &g);
}

// Brick of cells handled by one workgroup of the LJ kernels: the largest
// cube (3, 2 or 1 cells) whose tile at the mean occupancy fills at most 85%
// of the LDS tile ((B+2)^3 cells; with half lists the cells from the brick's
// first one on, of a smaller tile, at most 90%); workgroup size ~1.15x its
// particles.
void lj_grid(const mdpl_lj_params* p, Grid* g, int* threads) {
  int unit[3] = {1, 1, 1};
  make_grid(p->box, p->rc + p->skin, unit, g);
  const double per_cell = (double)p->n / ((double)g->nc[0] * g->nc[1] * g->nc[2]);
  int b = 1;
  for (int cand = 3; cand >= 1; --cand) {
    const bool half = p->pairs == MDPL_PAIRS_HALF;
    const int w = cand + 2, cells = half ? w * w * w - ((w + 1) * w + 1) : w * w * w;
    const double tile = cells * per_cell;
    if (half ? tile <= 0.9 * (kTileMaxHalf - 1) : tile <= 0.85 * kTileMax) {
      b = cand;
      break;
    }
  }
  int brick[3] = {b, b, b};
  make_grid(p->box, p->rc + p->skin, brick, g);
  int t = (int)(1.15 * g->V * per_cell + 0.5);
  t = ((t + 63) / 64) * 64;
  *threads = t < 64 ? 64 : (t > 1024 ? 1024 : t);
}

// Workgroups of any drifting launch: k_vv (256 particles each) or the fused
// force pass (the brick order, at most nbricks + 16 entries).
int64_t track_slots(int64_t n, const Grid& g) {
  const int64_t a = div_up(n, 256), b = (int64_t)g.nbricks + 16;
  return a > b ? a : b;
}

size_t lj_ws_bytes(const mdpl_lj_params* p, const Grid& g) {
  const int64_t n = p->n;
  const int64_t npad = div_up(n, 256) * 256;
  const size_t fb = p->precision == MDPL_FP32 ? 4 : 8;
  const int64_t nblk = div_up(n, 256) > g.nbricks ? div_up(n, 256) : g.nbricks;
  size_t b = sort_bytes(n);
  b += align256(4 * (size_t)(g.nkeys + 1));    // cell_start
  b += align256(4 * (size_t)n);                // perm
  b += 3 * align256(8 * (size_t)n);            // sx, sy, sz
  b += 3 * align256(8 * (size_t)n);            // avx..
  b += 3 * align256(fb * (size_t)n);           // afx..
  b += align256(4 * (size_t)n);                // aids
  b += 3 * align256(8 * (size_t)n);            // xb..
  b += 3 * align256(8 * (size_t)n);            // px..
  b += align256(2 * (size_t)((p->max_nb + 3) & ~3) * (size_t)npad);  // nbr (16-bit tile indices)
  b += align256(4 * (size_t)npad);             // cnt
  b += align256(4 * (size_t)kTabInts * (size_t)g.nbricks);  // tile tables
  b += align256(4 * (size_t)(g.nkeys + 1));                 // lower-x-half counts
  b += align256(4 * (size_t)(n + 1));          // offsets
  b += align256(8 * (size_t)(3 * nblk + 2));   // partials
  b += 2 * align256(8 * (size_t)track_slots(n, g));  // the rule's per-workgroup maxima
  b += align256(256);                          // flags, maxcount, max_disp, pe_w_tmp, rule, last row
  b += align256(4 * 8 * (size_t)g.nbricks);   // brick order of the tile kernels
  return b;
}

// The per-cell counts of the lower x half, when the list build may use them
// (full lists whose cells are wider than the list radius along x).
static int32_t* list_xlow(const mdpl_sim* s) { return s->tl.xlow; }

static bool thin_brick(const Grid& g, int b) {
  const int bx = b % g.nb[0], by = (b / g.nb[0]) % g.nb[1], bz = b / (g.nb[0] * g.nb[1]);
  return (bx == g.nb[0] - 1 && g.nc[0] % g.B[0]) || (by == g.nb[1] - 1 && g.nc[1] % g.B[1]) ||
         (bz == g.nb[2] - 1 && g.nc[2] % g.B[2]);
}

// The bricks of the 8 XCDs.  Workgroup w goes to XCD w mod 8 in dispatch
// order, so each round of 8 consecutive workgroups should carry equal work:
// the full bricks, in index order (z slowest), are dealt out in 8
// contiguous pieces (slabs of the box, whose tiles reload from the XCD's own
// L2), then the thin ones (the last brick along an axis whose cell count B
// does not divide) the same way, so that every XCD gets the same mix.
static std::vector<std::vector<int32_t>> xcd_bricks(const Grid& g) {
  std::vector<int32_t> full, thin;
  for (int b = 0; b < g.nbricks; ++b) (thin_brick(g, b) ? thin : full).push_back(b);
  std::vector<std::vector<int32_t>> xcd(8);
  for (const std::vector<int32_t>* v : {&full, &thin}) {
    const size_t per = (v->size() + 7) / 8;
    for (size_t k = 0; k < v->size(); ++k) xcd[k / per].push_back((*v)[k]);
  }
  return xcd;
}

// Workgroup -> brick of the tile kernels: workgroup w runs on XCD w mod 8;
// XCD x takes its bricks (xcd_bricks), the full ones first and then the thin
// ones, so that the light workgroups fill the last round.  8 entries per
// round; padding entries hold nbricks.
std::vector<int32_t> brick_order(const Grid& g) {
  const std::vector<std::vector<int32_t>> xcd = xcd_bricks(g);
  size_t most = 0;
  for (const auto& v : xcd) most = v.size() > most ? v.size() : most;
  std::vector<int32_t> order(most * 8, g.nbricks);
  for (int x = 0; x < 8; ++x)
    for (size_t j = 0; j < xcd[x].size(); ++j) order[j * 8 + x] = xcd[x][j];
  return order;
}

template <typename T>
T* take(char*& p, size_t bytes) {
  T* r = (T*)p;
  p += align256(bytes);
  return r;
}

double shift_value(const mdpl_lj_params* p) {
  if (p->shift == MDPL_SHIFT_PAPER) return p->eps;
  if (p->shift == MDPL_SHIFT_CUTOFF) {
    const double s2 = p->sigma * p->sigma / (p->rc * p->rc);
    const double s6 = s2 * s2 * s2;
    return -4.0 * p->eps * (s6 * s6 - s6);
  }
  return 0.0;
}

// An event from the pool (created only when the pool is empty).
// Whether this launch of the given kind is bracketed with events.
bool timed_launch(mdpl_sim* s, int slot) {
  if (!s->timing || slot < 0) return false;
  return (s->tm.launches[slot]++ % s->tm.every) == 0;
}

hipError_t take_event(mdpl_sim* s, hipEvent_t* e) {
  if (!s->tm.pool.empty()) {
    *e = s->tm.pool.back();
    s->tm.pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// kick (nullable): fuse the velocity-Verlet kick-kick-drift of the next step
// into the force pass (velocities of *kick updated, new positions to spare,
// KE of the sampled step to ke_dst); forces are then not stored.
mdpl_status launch_force(mdpl_sim* s, const double* x, const double* y, const double* z,
                         void* fx, void* fy, void* fz, const int32_t* scatter, bool energy,
                         double* e_atom, double* pe_w_dst, int kind, int timing_slot,
                         const StateArrays* kick = nullptr, double* const* spare = nullptr,
                         double* ke_dst = nullptr, double* disp_dst = nullptr) {
  ForceOut out;
  out.fx = fx;
  out.fy = fy;
  out.fz = fz;
  out.scatter = scatter;
  out.e_atom = e_atom;
  out.partials = s->partials;
  out.scale = 1.0;
  out.scale_dev = nullptr;
  out.fuse = kick != nullptr;
  out.vx = kick ? kick->vx : nullptr;
  out.vy = kick ? kick->vy : nullptr;
  out.vz = kick ? kick->vz : nullptr;
  out.nx = kick ? spare[0] : nullptr;
  out.ny = kick ? spare[1] : nullptr;
  out.nz = kick ? spare[2] : nullptr;
  out.h = s->p.dt / (2.0 * s->p.mass);
  out.dt = s->p.dt;
  out.flags = s->flags;
  out.track = s->track;
  if (!out.fuse) out.track.ring = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timed_launch(s, timing_slot)) {
    HIP_TRY(take_event(s, &e0));
    HIP_TRY(take_event(s, &e1));
    HIP_TRY(hipEventRecord(e0, s->st));
  }
  int nb = 0;
  HIP_TRY(lj_force(x, y, z, s->cell_start, s->g, s->tl, s->c, kind, energy, out, s->n, s->st, &nb));
  if (e1) {
    HIP_TRY(hipEventRecord(e1, s->st));
    s->tm.ev[timing_slot].push_back(e0);
    s->tm.ev[timing_slot].push_back(e1);
  }
  // PE, W (and the fused KE) of a sampled step, and the row's maximum
  // displacement (disp_dst), in one launch
  if (energy && pe_w_dst) {
    RowOut o{};
    o.dst[0] = pe_w_dst;
    o.dst[1] = pe_w_dst + 1;
    o.scale[0] = o.scale[1] = 1.0;
    int ncomp = 2;
    if (out.fuse && ke_dst) {
      o.dst[2] = ke_dst;
      o.scale[2] = 0.5 * s->p.mass;
      ncomp = 3;
    }
    if (disp_dst) {
      o.csrc = s->max_disp;
      o.cdst = disp_dst;
    }
    HIP_TRY(reduce_row(s->partials, nb, out.fuse ? 3 : 2, ncomp, o, s->st));
  }
  return MDPL_OK;
}

}  // namespace

extern "C" {

mdpl_status mdpl_workspace_bytes(const mdpl_lj_params* p, size_t* bytes) {
  if (!bytes) return MDPL_EINVAL;
  mdpl_status v = validate(p);
  if (v != MDPL_OK) return v;
  Grid g;
  int threads;
  lj_grid(p, &g, &threads);
  *bytes = lj_ws_bytes(p, g);
  return MDPL_OK;
}

mdpl_status mdpl_sim_create(const mdpl_lj_params* p, void* workspace, size_t bytes, void* stream,
                            mdpl_sim** out) {
  if (!out || !workspace) return MDPL_EINVAL;
  mdpl_status v = validate(p);
  if (v != MDPL_OK) return v;
  if (((uintptr_t)workspace & 255) != 0) return MDPL_EWORKSPACE;
  mdpl_sim* s = new (std::nothrow) mdpl_sim();
  if (!s) return MDPL_EINVAL;
  s->p = *p;
  s->st = (hipStream_t)stream;
  int threads = 64;
  lj_grid(p, &s->g, &threads);
  if (bytes < lj_ws_bytes(p, s->g)) {
    delete s;
    return MDPL_EWORKSPACE;
  }
  s->n = p->n;
  s->npad = div_up(p->n, 256) * 256;
  const double rext = p->rc + p->skin;
  s->r2ext = rext * rext;
  s->fbytes = p->precision == MDPL_FP32 ? 4 : 8;
  s->c.rc2 = p->rc * p->rc;
  s->c.eps = p->eps;
  s->c.sigma2 = p->sigma * p->sigma;
  s->c.shift_v = shift_value(p);
  for (int k = 0; k < 3; ++k) {
    s->c.box[k] = p->box[k];
    s->c.half[k] = 0.5 * p->box[k];
    s->c.inv_box[k] = 1.0 / p->box[k];
  }
  const int64_t n = s->n;
  char* w = (char*)workspace;
  sort_carve(w, n, &s->sort);
  s->cell_start = take<int32_t>(w, 4 * (size_t)(s->g.nkeys + 1));
  s->perm = take<int32_t>(w, 4 * (size_t)n);
  s->sx = take<double>(w, 8 * (size_t)n);
  s->sy = take<double>(w, 8 * (size_t)n);
  s->sz = take<double>(w, 8 * (size_t)n);
  s->avx = take<double>(w, 8 * (size_t)n);
  s->avy = take<double>(w, 8 * (size_t)n);
  s->avz = take<double>(w, 8 * (size_t)n);
  s->afx = take<char>(w, s->fbytes * (size_t)n);
  s->afy = take<char>(w, s->fbytes * (size_t)n);
  s->afz = take<char>(w, s->fbytes * (size_t)n);
  s->aids = take<int32_t>(w, 4 * (size_t)n);
  s->xb = take<double>(w, 8 * (size_t)n);
  s->yb = take<double>(w, 8 * (size_t)n);
  s->zb = take<double>(w, 8 * (size_t)n);
  s->px = take<double>(w, 8 * (size_t)n);
  s->py = take<double>(w, 8 * (size_t)n);
  s->pz = take<double>(w, 8 * (size_t)n);
  const int max_nb4 = (p->max_nb + 3) & ~3;
  s->tl.nbr = take<uint64_t>(w, 2 * (size_t)max_nb4 * (size_t)s->npad);
  s->tl.cnt = take<int32_t>(w, 4 * (size_t)s->npad);
  s->tl.tab = take<int32_t>(w, 4 * (size_t)kTabInts * (size_t)s->g.nbricks);
  s->tl.stride = s->npad;
  s->tl.max_nb = p->max_nb;
  s->tl.half = p->pairs == MDPL_PAIRS_HALF;
  s->tl.cells = p->pairs == MDPL_PAIRS_CELLS;
  s->tl.threads = threads;
  s->tl.xlow = take<int32_t>(w, 4 * (size_t)(s->g.nkeys + 1));
  // a particle's far half of the next cell along x lies beyond the list
  // radius only if the cell is wider than that radius (with room for the
  // rounding of the FP64 test)
  if (s->tl.half || s->tl.cells || !(p->box[0] / s->g.nc[0] > rext * (1.0 + 1e-9)))
    s->tl.xlow = nullptr;
  s->offsets = take<int32_t>(w, 4 * (size_t)(n + 1));
  s->nblk = (int)(div_up(n, 256) > s->g.nbricks ? div_up(n, 256) : s->g.nbricks);
  s->partials = take<double>(w, 8 * (size_t)(3 * s->nblk + 2));
  s->nvpart = (int)track_slots(n, s->g);
  s->vpart[0] = take<double>(w, 8 * (size_t)s->nvpart);
  s->vpart[1] = take<double>(w, 8 * (size_t)s->nvpart);
  char* small = take<char>(w, 256);
  {
    const std::vector<int32_t> order = brick_order(s->g);
    int32_t* dorder = take<int32_t>(w, 4 * 8 * (size_t)s->g.nbricks);
    const hipError_t e = hipMemcpy(dorder, order.data(), 4 * order.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      g_last_hip_error = (int32_t)e;
      delete s;
      return MDPL_EHIP;
    }
    s->g.order = dorder;
    s->g.norder = (int)order.size();
  }
  s->flags = (uint32_t*)small;
  s->maxcount = (int32_t*)(small + 4);
  s->max_disp = (double*)(small + 8);
  s->pe_w_tmp = (double*)(small + 16);
  s->bound = (double*)(small + 48);
  s->last_row = (double*)(small + 64);
  s->built = false;
  s->have_list = false;
  s->timing = false;
  s->resume.valid = false;
  s->gstep = s->kb = s->since = 0;
  s->have_ref = false;
  s->last_row_valid = false;
  s->n_rebuilds = s->n_early = s->n_syncs = 0;
  s->ring_host = s->ring_dev = nullptr;
  {
    // the rule's records: pinned host memory the kernels write through
    void* h = nullptr;
    hipError_t e = hipHostMalloc(&h, sizeof(KickRecord) * kRing,
                                 hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) {
      memset(h, 0, sizeof(KickRecord) * kRing);
      for (int q = 0; q < kRing; ++q) ((KickRecord*)h)[q].stamp = -1;
      e = hipHostGetDevicePointer((void**)&s->ring_dev, h, 0);
    }
    if (e != hipSuccess) {
      if (h) (void)hipHostFree(h);
      g_last_hip_error = (int32_t)e;
      delete s;
      return MDPL_EHIP;
    }
    s->ring_host = (KickRecord*)h;
  }
  s->track = KickTrack{};
  s->track.part[0] = s->vpart[0];
  s->track.part[1] = s->vpart[1];
  s->track.bound = s->bound;
  s->track.dt = p->dt;
  s->pend_n = 0;
  s->pend_step = 0;
  s->track_cur = 0;
  hipError_t e = hipMemsetAsync(small, 0, 256, s->st);
  if (e != hipSuccess) {
    g_last_hip_error = (int32_t)e;
    (void)hipHostFree(s->ring_host);
    delete s;
    return MDPL_EHIP;
  }
  *out = s;
  return MDPL_OK;
}

mdpl_status mdpl_sim_destroy(mdpl_sim* s) {
  if (!s) return MDPL_EINVAL;
  // the kernels may still write the records: finish the stream first
  (void)hipStreamSynchronize(s->st);
  for (int k = 0; k < 2; ++k)
    for (hipEvent_t e : s->tm.ev[k]) (void)hipEventDestroy(e);
  for (hipEvent_t e : s->tm.pool) (void)hipEventDestroy(e);
  if (s->ring_host) (void)hipHostFree(s->ring_host);
  delete s;
  return MDPL_OK;
}

mdpl_status mdpl_build(mdpl_sim* s, const double* x, const double* y, const double* z) {
  if (!s || !x || !y || !z) return MDPL_EINVAL;
  s->resume.valid = false;
  int32_t *skeys, *svals;
  HIP_TRY(bin_particles(x, y, z, s->n, s->g, s->sort, s->cell_start, &skeys, &svals, s->st,
                        list_xlow(s)));
  HIP_TRY(hipMemcpyAsync(s->perm, svals, 4 * (size_t)s->n, hipMemcpyDeviceToDevice, s->st));
  s->skeys = skeys;
  HIP_TRY(gather_positions(x, y, z, s->perm, s->n, s->sx, s->sy, s->sz, s->p.box, true, s->st));
  if (!s->tl.cells)
    HIP_TRY(build_tile_nlist(s->sx, s->sy, s->sz, skeys, s->cell_start, s->g, s->r2ext, s->tl,
                             s->flags, s->maxcount, s->st));
  s->built = true;
  s->have_list = !s->tl.cells;
  s->resume.valid = false;  // the list of the last run is overwritten
  return MDPL_OK;
}

mdpl_status mdpl_nlist_export(mdpl_sim* s, int32_t* i_out, int32_t* j_out, int64_t cap,
                              int64_t* count_host) {
  if (!s || !count_host || cap < 0 || (cap > 0 && (!i_out || !j_out))) return MDPL_EINVAL;
  if (!s->built || s->tl.cells) return MDPL_ESTATE;
  HIP_TRY(exclusive_scan(s->tl.cnt, s->offsets, s->n, s->sort.blocksums, true, s->st));
  if (cap > 0)
    HIP_TRY(export_tile_pairs(s->tl, s->cell_start, s->g, s->perm, s->offsets, i_out, j_out, cap,
                              s->st));
  int32_t total = 0;
  HIP_TRY(hipMemcpyAsync(&total, s->offsets + s->n, 4, hipMemcpyDeviceToHost, s->st));
  HIP_TRY(hipStreamSynchronize(s->st));
  *count_host = total;
  return MDPL_OK;
}

mdpl_status mdpl_nlist_entries(mdpl_sim* s, int64_t* entries) {
  if (!s || !entries) return MDPL_EINVAL;
  if (!s->have_list) return MDPL_ESTATE;
  HIP_TRY(exclusive_scan(s->tl.cnt, s->offsets, s->n, s->sort.blocksums, true, s->st));
  int32_t total = 0;
  HIP_TRY(hipMemcpyAsync(&total, s->offsets + s->n, 4, hipMemcpyDeviceToHost, s->st));
  HIP_TRY(hipStreamSynchronize(s->st));
  *entries = total;
  return MDPL_OK;
}

mdpl_status mdpl_forces(mdpl_sim* s, const double* x, const double* y, const double* z, void* fx,
                        void* fy, void* fz, double* pe_w, double* e_atom) {
  if (!s || !x || !y || !z || !fx || !fy || !fz) return MDPL_EINVAL;
  if (!s->built) return MDPL_ESTATE;
  HIP_TRY(gather_canonical(x, y, z, s->perm, s->skeys, s->n, s->g, s->sx, s->sy, s->sz, s->st));
  const bool energy = pe_w != nullptr || e_atom != nullptr;
  return launch_force(s, s->sx, s->sy, s->sz, fx, fy, fz, s->perm, energy, e_atom, pe_w,
                      s->p.precision, -1);
}

mdpl_status mdpl_lj_backward(mdpl_sim* s, const double* x, const double* y, const double* z,
                             const double* grad_e, double* gx, double* gy, double* gz) {
  if (!s || !x || !y || !z || !grad_e || !gx || !gy || !gz) return MDPL_EINVAL;
  if (!s->built) return MDPL_ESTATE;
  HIP_TRY(gather_canonical(x, y, z, s->perm, s->skeys, s->n, s->g, s->sx, s->sy, s->sz, s->st));
  ForceOut out;
  out.fx = gx;
  out.fy = gy;
  out.fz = gz;
  out.scatter = s->perm;
  out.e_atom = nullptr;
  out.partials = s->partials;
  out.scale = -1.0;
  out.scale_dev = grad_e;
  out.fuse = false;
  out.flags = s->flags;
  // FP64 arithmetic for the FP64 context, FP32 pair math for the FP32 one;
  // the gradient is stored in double either way
  const int kind = s->p.precision == MDPL_FP64 ? 2 : 3;
  HIP_TRY(lj_force(s->sx, s->sy, s->sz, s->cell_start, s->g, s->tl, s->c, kind, false, out, s->n, s->st,
                   nullptr));
  return MDPL_OK;
}

mdpl_status mdpl_check(mdpl_sim* s, uint32_t* flags_host, int32_t* max_count_host) {
  if (!s) return MDPL_EINVAL;
  uint32_t f = 0;
  int32_t m = 0;
  HIP_TRY(hipMemcpyAsync(&f, s->flags, 4, hipMemcpyDeviceToHost, s->st));
  HIP_TRY(hipMemcpyAsync(&m, s->maxcount, 4, hipMemcpyDeviceToHost, s->st));
  HIP_TRY(hipStreamSynchronize(s->st));
  if (flags_host) *flags_host = f;
  if (max_count_host) *max_count_host = m;
  if (f & MDPL_FLAG_NL_OVERFLOW) return MDPL_ECAPACITY;
  if (f & MDPL_FLAG_SKIN) return MDPL_ESKIN;
  if (f & MDPL_FLAG_NONFINITE) return MDPL_ENONFINITE;
  return MDPL_OK;
}

mdpl_status mdpl_clear_flags(mdpl_sim* s) {
  if (!s) return MDPL_EINVAL;
  HIP_TRY(hipMemsetAsync(s->flags, 0, 16, s->st));
  return MDPL_OK;
}

mdpl_status mdpl_set_timing(mdpl_sim* s, int32_t on, int32_t every) {
  if (!s || on < 0 || every < 1) return MDPL_EINVAL;
  s->timing = on != 0;
  s->tm.every = every;
  s->tm.launches[0] = s->tm.launches[1] = 0;
  // reserve event pairs so that no event is created while timing
  const size_t want = on > 1 ? 4 * (size_t)on : 0;
  while (s->tm.pool.size() < want) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    s->tm.pool.push_back(e);
  }
  return MDPL_OK;
}

mdpl_status mdpl_kernel_time(mdpl_sim* s, int32_t which, double* ms, int64_t* launches) {
  if (!s || which < 0 || which > 1) return MDPL_EINVAL;
  HIP_TRY(hipStreamSynchronize(s->st));
  double tot = 0.0;
  std::vector<hipEvent_t>& v = s->tm.ev[which];
  for (size_t k = 0; k + 1 < v.size(); k += 2) {
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, v[k], v[k + 1]));
    tot += t;
  }
  if (ms) *ms = tot;
  if (launches) *launches = (int64_t)(v.size() / 2);
  for (hipEvent_t e : v) s->tm.pool.push_back(e);
  v.clear();
  s->tm.launches[which] = 0;
  return MDPL_OK;
}

mdpl_status mdpl_rebuild_stats(mdpl_sim* s, int64_t* rebuilds, int64_t* early, int64_t* syncs) {
  if (!s) return MDPL_EINVAL;
  if (rebuilds) *rebuilds = s->n_rebuilds;
  if (early) *early = s->n_early;
  if (syncs) *syncs = s->n_syncs;
  return MDPL_OK;
}

}  // extern "C"

namespace {

// One record of the rule's ring, read consistently (the stamp before and
// after the fields); false if the device was writing it.
bool read_record(const KickRecord* p, KickRecord* out) {
  const int64_t a = __atomic_load_n(&p->stamp, __ATOMIC_ACQUIRE);
  out->bound = ((const volatile KickRecord*)p)->bound;
  out->vmax = ((const volatile KickRecord*)p)->vmax;
  __atomic_thread_fence(__ATOMIC_ACQUIRE);
  const int64_t b = __atomic_load_n(&p->stamp, __ATOMIC_ACQUIRE);
  out->stamp = a;
  return a == b && a >= 0;
}

// The newest record the device has published (stamp <= upto) and the largest
// speed of all records in the ring.
bool latest_record(const mdpl_sim* s, int64_t upto, KickRecord* out, double* vref) {
  bool have = false;
  *vref = 0.0;
  for (int q = 0; q < kRing; ++q) {
    KickRecord r;
    if (!read_record(s->ring_host + q, &r) || r.stamp > upto) continue;
    *vref = r.vmax > *vref ? r.vmax : *vref;
    if (!have || r.stamp > out->stamp) {
      *out = r;
      have = true;
    }
  }
  return have;
}

// Waits (without draining the stream) until the device has published the
// record of step `target` or a later one.
mdpl_status wait_record(mdpl_sim* s, int64_t target) {
  for (int64_t it = 0;; ++it) {
    KickRecord r;
    double v;
    if (latest_record(s, INT64_MAX, &r, &v) && r.stamp >= target) return MDPL_OK;
    if ((it & 1023) == 1023) {
      const hipError_t q = hipStreamQuery(s->st);
      if (q == hipSuccess) return MDPL_OK;  // idle: nothing more will come
      (void)hipGetLastError();              // a not-ready query is not an error of the library
      if (q != hipErrorNotReady) {
        g_last_hip_error = (int32_t)q;
        return MDPL_EHIP;
      }
    }
    std::this_thread::yield();
  }
}

// The rebuild rule of Eq. extended_cutoff for the positions of step k =
// s->gstep: rebuild when 2 * bound >= skin, bound = sum over the steps since
// the last build of dt * max|v| (the device's records).  The host predicts
// the bound from the newest record it can see, allowing the largest recent
// speed to double in the steps it cannot see yet; only when that prediction
// reaches the threshold does it wait for the stream and decide on the exact
// record of step k.  So the rebuilds are those of the rule itself, unless a
// speed more than doubles within the host's lag (the displacement check at
// every rebuild still flags a list used too long).
mdpl_status rule_decide(mdpl_sim* s, bool* need) {
  const int64_t k = s->gstep;
  const double dt = s->p.dt, skin = s->p.skin;
  KickRecord r;
  double vref = 0.0;
  bool have = latest_record(s, k, &r, &vref);
  if (have && k - r.stamp > kLagMax) {
    const mdpl_status e = wait_record(s, k - kLagKeep);
    if (e != MDPL_OK) return e;
    have = latest_record(s, k, &r, &vref);
  }
  if (have) {
    const double base = r.stamp > s->kb ? r.bound : 0.0;
    const int64_t from = r.stamp > s->kb ? r.stamp : s->kb;
    const double pred = base + (double)(k - from) * dt * (kSpeedHeadroom * vref);
    if (2.0 * pred < skin) {
      *need = false;
      return MDPL_OK;
    }
  }
  if (s->pend_n > 0) {  // the record of step k is still pending: publish it now
    KickTrack kt = s->track;
    kt.cur = s->track_cur;
    kt.pub_n = s->pend_n;
    kt.pub_step = s->pend_step;
    HIP_TRY(publish_record(kt, s->st));
    s->pend_n = 0;
  }
  HIP_TRY(hipStreamSynchronize(s->st));
  ++s->n_syncs;
  KickRecord rk;
  if (!read_record(s->ring_host + (k & (kRing - 1)), &rk) || rk.stamp != k) {
    *need = true;  // no record of this step: rebuild to be safe
    return MDPL_OK;
  }
  *need = 2.0 * rk.bound >= skin;
  return MDPL_OK;
}

bool same_arrays(const StateArrays& a, const StateArrays& b) {
  return a.x == b.x && a.y == b.y && a.z == b.z && a.vx == b.vx && a.vy == b.vy && a.vz == b.vz &&
         a.fx == b.fx && a.fy == b.fy && a.fz == b.fz && a.ids == b.ids;
}

// The time loop of Alg. VelocityVerlet with list reuse (Sec. 3.5), shared by
// the LJ and learned-potential runs.  force(cur, energy, pe_w_dst, slot, fuse,
// spare, ke_dst, disp_dst) fills cur.f* from cur positions (on sampled steps
// also PE, W into pe_w_dst and the maximum displacement since the last build
// into disp_dst); with fuse it also applies the next step's kick-kick-drift,
// the new positions going to spare.
// th (nullable): Andersen collisions after every completed step; global
// step numbers start at th->step (the step0 of mdpl_run_andersen) + 1.
// start: MDPL_RUN_SETUP bins, builds and computes F(r0) first;
// MDPL_RUN_CONTINUE takes over the state that the last run of this kind left
// in the same arrays (list, forces, step count since the build).
// Positions are double-buffered (the drift writes to the spare buffer), so
// that at a rebuild the positions of the last force pass with the old list
// are still there for the displacement check.
template <typename ForceFn>
mdpl_status run_loop(mdpl_sim* s, StateArrays user, int64_t nsteps, int32_t sample_every,
                     double* thermo, bool can_fuse, ForceFn force, int kind, int32_t start,
                     const Andersen* th = nullptr) {
  if (start != MDPL_RUN_SETUP && start != MDPL_RUN_CONTINUE) return MDPL_EINVAL;
  const bool cont = start == MDPL_RUN_CONTINUE;
  if (cont && !(s->resume.valid && s->resume.kind == kind && same_arrays(s->resume.arrays, user)))
    return MDPL_ESTATE;
  s->resume.valid = false;  // until this run has been enqueued completely
  const int64_t n = s->n;
  const int prec = s->p.precision;
  const int ns = s->p.reuse_every;
  const double dt = s->p.dt;
  const double h = dt / (2.0 * s->p.mass);
  const double half_skin = 0.5 * s->p.skin;
  const double ke_scale = 0.5 * s->p.mass;
  const bool rule = s->p.rebuild == MDPL_REBUILD_VMAX;
  StateArrays alt{s->sx, s->sy, s->sz, s->avx, s->avy, s->avz, s->afx, s->afy, s->afz, s->aids};
  StateArrays cur = user, other = alt;
  double* spare[3] = {s->px, s->py, s->pz};
  Andersen thermo_cfg{};
  s->built = false;  // the standalone build is overwritten
  s->track.ring = rule ? s->ring_dev : nullptr;

  // check: the displacement of the last force pass with the old list (in
  // spare, the drift's other buffer) against half the skin
  auto rebuild = [&](bool check, bool early) -> mdpl_status {
    if (check && s->have_ref) {
      int nb = 0;
      HIP_TRY(disp_partials(spare[0], spare[1], spare[2], s->xb, s->yb, s->zb, n, s->partials,
                            s->st, &nb));
      HIP_TRY(skin_check(s->partials, nb, half_skin, s->max_disp, s->flags, s->st));
    }
    int32_t *skeys, *svals;
    HIP_TRY(bin_particles(cur.x, cur.y, cur.z, n, s->g, s->sort, s->cell_start, &skeys, &svals,
                          s->st, list_xlow(s)));
    HIP_TRY(reorder_state(cur, svals, n, s->fbytes, s->p.box, other, s->xb, s->yb, s->zb,
                          s->bound, s->st));
    StateArrays t = cur;
    cur = other;
    other = t;
    if (!s->tl.cells)
      HIP_TRY(build_tile_nlist(cur.x, cur.y, cur.z, skeys, s->cell_start, s->g, s->r2ext, s->tl,
                               s->flags, s->maxcount, s->st));
    s->have_ref = true;
    s->have_list = !s->tl.cells;
    s->pend_n = 0;  // bound restarts at zero with the new list
    s->kb = s->gstep;
    s->since = 0;
    ++s->n_rebuilds;
    if (early) ++s->n_early;
    return MDPL_OK;
  };
  auto row = [&](int64_t step) { return thermo + 4 * (step / sample_every); };
  auto sampled = [&](int64_t step) { return sample_every > 0 && step % sample_every == 0; };
  auto swap_positions = [&]() {
    double* t[3] = {cur.x, cur.y, cur.z};
    cur.x = spare[0];
    cur.y = spare[1];
    cur.z = spare[2];
    spare[0] = t[0];
    spare[1] = t[1];
    spare[2] = t[2];
  };

  // the rule's bookkeeping around every drifting launch (no-op without the rule)
  auto arm = [&]() {
    s->track.step = s->gstep + 1;
    s->track.cur = s->track_cur;
    s->track.pub_n = s->pend_n;
    s->track.pub_step = s->pend_step;
  };
  auto drifted = [&](int groups) {
    if (!s->track.ring) return;
    s->pend_n = groups;
    s->pend_step = s->track.step;
    s->track_cur ^= 1;
  };
  const int force_groups = s->g.order ? s->g.norder : ((s->g.nbricks + 7) / 8) * 8;

  mdpl_status r = MDPL_OK;
  if (!cont) {
    r = rebuild(false, false);
    if (r != MDPL_OK) return r;
    r = force(cur, sampled(0), sampled(0) ? row(0) + 1 : nullptr, -1, false, spare, nullptr,
              sampled(0) ? row(0) + 3 : nullptr);
    if (r != MDPL_OK) return r;
  } else if (sampled(0) && s->last_row_valid) {
    // the positions are the last run's final ones, whose PE, W it sampled
    // (the KE is formed again below: velocities may have been rescaled)
    HIP_TRY(hipMemcpyAsync(row(0), s->last_row, 4 * sizeof(double), hipMemcpyDeviceToDevice, s->st));
  } else if (sampled(0)) {
    // PE, W of the current state from a pass whose forces go to scratch
    StateArrays tmp = cur;
    tmp.fx = other.fx;
    tmp.fy = other.fy;
    tmp.fz = other.fz;
    r = force(tmp, true, row(0) + 1, -1, false, spare, nullptr, row(0) + 3);
    if (r != MDPL_OK) return r;
  }
  if (sampled(0)) {
    int nb = 0;
    HIP_TRY(vv_step(cur.x, cur.y, cur.z, nullptr, nullptr, nullptr, cur.vx, cur.vy, cur.vz,
                    cur.fx, cur.fy, cur.fz, prec, n, h, dt, 3, true, s->partials, s->flags, s->st,
                    &nb));
    HIP_TRY(reduce_partials(s->partials, nb, 1, 1, row(0), ke_scale, s->st));
  }
  // the collisions at the end of global step g (the kick completing it is in vv_step)
  auto collide = [&](int64_t local) -> const Andersen* {
    if (!th) return nullptr;
    thermo_cfg = *th;
    thermo_cfg.ids = cur.ids;
    thermo_cfg.step = th->step + local;
    return &thermo_cfg;
  };
  bool fused = false;  // the last force pass already applied this step's kick-kick-drift
  for (int64_t step = 1; step <= nsteps; ++step) {
    if (!fused) {
      const bool ke = step > 1 && sampled(step - 1);
      int nb = 0;
      arm();
      HIP_TRY(vv_step(cur.x, cur.y, cur.z, spare[0], spare[1], spare[2], cur.vx, cur.vy, cur.vz,
                      cur.fx, cur.fy, cur.fz, prec, n, h, dt, step == 1 ? 0 : 1, ke, s->partials,
                      s->flags, s->st, &nb, step == 1 ? nullptr : collide(step - 1), &s->track));
      drifted(nb);
      swap_positions();
      if (ke) HIP_TRY(reduce_partials(s->partials, nb, 1, 1, row(step - 1), ke_scale, s->st));
    }
    ++s->gstep;
    ++s->since;
    bool need = s->since >= ns, early = false;
    if (!need && rule) {
      r = rule_decide(s, &need);
      if (r != MDPL_OK) return r;
      early = need;
    }
    if (need) {
      r = rebuild(true, early);
      if (r != MDPL_OK) return r;
    }
    const bool en = sampled(step);
    // the pass of the last step stores its forces for the final half kick
    fused = can_fuse && step < nsteps;
    if (fused) arm();
    r = force(cur, en, en ? row(step) + 1 : nullptr, en ? 1 : 0, fused, spare,
              en ? row(step) : nullptr, en ? row(step) + 3 : nullptr);
    if (r != MDPL_OK) return r;
    if (fused) {
      drifted(force_groups);
      swap_positions();
    }
  }
  if (nsteps > 0) {
    const bool ke = sampled(nsteps);
    int nb = 0;
    HIP_TRY(vv_step(cur.x, cur.y, cur.z, nullptr, nullptr, nullptr, cur.vx, cur.vy, cur.vz,
                    cur.fx, cur.fy, cur.fz, prec, n, h, dt, 2, ke, s->partials, s->flags, s->st,
                    &nb, collide(nsteps)));
    if (ke) HIP_TRY(reduce_partials(s->partials, nb, 1, 1, row(nsteps), ke_scale, s->st));
    // close the last reuse period: the final positions were used by the last pass
    HIP_TRY(disp_partials(cur.x, cur.y, cur.z, s->xb, s->yb, s->zb, n, s->partials, s->st, &nb));
    HIP_TRY(skin_check(s->partials, nb, half_skin, s->max_disp, s->flags, s->st));
  }
  // the state ends wherever the ping-pong left it: copy back what is not in the caller's arrays
  HIP_TRY(copy_state(cur, user, n, s->fbytes, s->st));
  s->last_row_valid = sampled(nsteps);
  if (s->last_row_valid)
    HIP_TRY(hipMemcpyAsync(s->last_row, row(nsteps), 4 * sizeof(double), hipMemcpyDeviceToDevice,
                           s->st));
  s->resume.valid = true;
  s->resume.kind = kind;
  s->resume.arrays = user;
  return MDPL_OK;
}

}  // namespace

extern "C" {

mdpl_status mdpl_run(mdpl_sim* s, double* x, double* y, double* z, double* vx, double* vy,
                     double* vz, void* fx, void* fy, void* fz, int32_t* ids, int64_t nsteps,
                     int32_t sample_every, double* thermo, int32_t start) {
  if (!s || !x || !y || !z || !vx || !vy || !vz || !fx || !fy || !fz || !ids) return MDPL_EINVAL;
  if (nsteps < 0 || sample_every < 0 || (sample_every > 0 && !thermo)) return MDPL_EINVAL;
  const int prec = s->p.precision;
  StateArrays user{x, y, z, vx, vy, vz, fx, fy, fz, ids};
  // the kicks are fused into the full-list pass only (a half-list force is
  // complete only when its pass has ended; the cell pass has no fused form)
  return run_loop(s, user, nsteps, sample_every, thermo, !s->tl.half && !s->tl.cells,
                  [&](const StateArrays& cur, bool en, double* pe_w, int slot, bool fuse,
                      double* const* spare, double* ke, double* disp) {
                    return launch_force(s, cur.x, cur.y, cur.z, cur.fx, cur.fy, cur.fz, nullptr,
                                        en, nullptr, pe_w, prec, slot, fuse ? &cur : nullptr,
                                        spare, ke, disp);
                  },
                  kKindLJ, start);
}

mdpl_status mdpl_run_andersen(mdpl_sim* s, double* x, double* y, double* z, double* vx,
                              double* vy, double* vz, void* fx, void* fy, void* fz, int32_t* ids,
                              int64_t nsteps, int32_t sample_every, double* thermo,
                              double temperature, double collision_rate, uint64_t seed,
                              int64_t step0, int32_t start) {
  if (!s || !x || !y || !z || !vx || !vy || !vz || !fx || !fy || !fz || !ids) return MDPL_EINVAL;
  if (nsteps < 0 || sample_every < 0 || (sample_every > 0 && !thermo) || step0 < 0) return MDPL_EINVAL;
  const double p = collision_rate * s->p.dt;
  if (!(temperature >= 0.0) || !isfinite(temperature) || !(collision_rate >= 0.0) || !(p <= 1.0))
    return MDPL_EINVAL;
  const int prec = s->p.precision;
  const Andersen th{nullptr, p, sqrt(temperature / s->p.mass), seed, step0};
  StateArrays user{x, y, z, vx, vy, vz, fx, fy, fz, ids};
  // the collisions sit between the kicks of vv_step: no fused kicks
  return run_loop(
      s, user, nsteps, sample_every, thermo, false,
      [&](const StateArrays& cur, bool en, double* pe_w, int slot, bool, double* const*, double*,
          double* disp) {
        return launch_force(s, cur.x, cur.y, cur.z, cur.fx, cur.fy, cur.fz, nullptr, en, nullptr,
                            pe_w, prec, slot, nullptr, nullptr, nullptr, disp);
      },
      kKindLJ, start, &th);
}

// ------------------------------------------------------------ analysis
static size_t analysis_bytes(int64_t n, const Grid& g, int max_nb) {
  size_t b = sort_bytes(n);
  b += align256(4 * (size_t)(g.nkeys + 1));
  b += align256(4 * (size_t)n);          // perm
  b += 3 * align256(8 * (size_t)n);      // sorted positions
  b += align256(4 * (size_t)n * (size_t)max_nb);
  b += align256(4 * (size_t)n);          // cnt
  b += align256(64);
  return b;
}

static mdpl_status analysis_prep(const double* x, const double* y, const double* z, int64_t n,
                                 const double* box, double rc, int max_nb, void* ws, size_t bytes,
                                 hipStream_t st, Grid* g, SortBufs* sb, int32_t** cs,
                                 int32_t** perm, double** sx, double** sy, double** sz,
                                 int32_t** skeys, NList* nl, uint32_t** small) {
  if (!x || !y || !z || !box || !ws || n <= 0 || n > (1ll << 26)) return MDPL_EINVAL;
  if (!(rc > 0.0) || !isfinite(rc) || max_nb < 1 || max_nb > 1024) return MDPL_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (!(box[k] > 0.0) || !isfinite(box[k])) return MDPL_EINVAL;
  if (((uintptr_t)ws & 255) != 0) return MDPL_EWORKSPACE;
  int unit[3] = {1, 1, 1};
  mdpl_status v = make_grid(box, rc, unit, g);
  if (v != MDPL_OK) return v;
  if (bytes < analysis_bytes(n, *g, max_nb)) return MDPL_EWORKSPACE;
  char* w = (char*)ws;
  sort_carve(w, n, sb);
  *cs = take<int32_t>(w, 4 * (size_t)(g->nkeys + 1));
  *perm = take<int32_t>(w, 4 * (size_t)n);
  *sx = take<double>(w, 8 * (size_t)n);
  *sy = take<double>(w, 8 * (size_t)n);
  *sz = take<double>(w, 8 * (size_t)n);
  nl->nbr = take<int32_t>(w, 4 * (size_t)n * (size_t)max_nb);
  nl->cnt = take<int32_t>(w, 4 * (size_t)n);
  nl->stride = n;
  nl->max_nb = max_nb;
  nl->layout = 1;
  *small = take<uint32_t>(w, 64);
  int32_t* svals;
  HIP_TRY(bin_particles(x, y, z, n, *g, *sb, *cs, skeys, &svals, st));
  HIP_TRY(hipMemcpyAsync(*perm, svals, 4 * (size_t)n, hipMemcpyDeviceToDevice, st));
  HIP_TRY(gather_positions(x, y, z, *perm, n, *sx, *sy, *sz, box, false, st));
  return MDPL_OK;
}

mdpl_status mdpl_analysis_workspace_bytes(int64_t n, const double* box, double rc, int32_t max_nb,
                                          size_t* bytes) {
  if (!box || !bytes || n <= 0 || n > (1ll << 26) || !(rc > 0.0) || max_nb < 1 || max_nb > 1024)
    return MDPL_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (!(box[k] > 0.0) || !isfinite(box[k])) return MDPL_EINVAL;
  Grid g;
  int unit[3] = {1, 1, 1};
  mdpl_status v = make_grid(box, rc, unit, &g);
  if (v != MDPL_OK) return v;
  *bytes = analysis_bytes(n, g, max_nb);
  return MDPL_OK;
}

// Scratch of mdpl_boa_noalloc: a static device array (each GPU holds its
// own copy), whose device address is looked up once per device with that
// device current; host code uses only that address, never the array's name.
static __device__ __align__(256) unsigned char scratch[MDPL_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_dev[256];

static mdpl_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    g_last_hip_error = (int32_t)e;
    return MDPL_EHIP;
  }
  if (dev < 0 || dev >= 256) return MDPL_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      g_last_hip_error = (int32_t)(e != hipSuccess ? e : hipErrorInvalidSymbol);
      return MDPL_EHIP;
    }
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return MDPL_OK;
}

mdpl_status mdpl_boa(const double* x, const double* y, const double* z, int64_t n,
                     const double* box, double rc, float* q4, float* q5, float* q6, int32_t* nnb,
                     void* ws, size_t bytes, void* stream) {
  if (!q4 || !q6 || !nnb) return MDPL_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  Grid g;
  SortBufs sb;
  int32_t *cs, *perm, *skeys;
  double *sx, *sy, *sz;
  NList nl;
  uint32_t* small;
  // the bond-order pass walks the cells itself: no list is stored
  mdpl_status v = analysis_prep(x, y, z, n, box, rc, 1, ws, bytes, st, &g, &sb, &cs, &perm, &sx,
                                &sy, &sz, &skeys, &nl, &small);
  if (v != MDPL_OK) return v;
  HIP_TRY(boa_q(sx, sy, sz, skeys, cs, perm, n, g, rc * rc, q4, q5, q6, nnb, st));
  return MDPL_OK;
}

mdpl_status mdpl_boa_noalloc(const double* x, const double* y, const double* z, int64_t n,
                             const double* box, double rc, float* q4, float* q5, float* q6,
                             int32_t* nnb, void* stream) {
  size_t need = 0;
  mdpl_status v = mdpl_analysis_workspace_bytes(n, box, rc, 1, &need);
  if (v != MDPL_OK) return v;
  if (need > (size_t)MDPL_SCRATCH_BYTES) return MDPL_ESCRATCH;
  void* ws = nullptr;
  v = scratch_address(&ws);
  if (v != MDPL_OK) return v;
  // the bond-order pass writes every scratch word it reads (no clearing needed)
  return mdpl_boa(x, y, z, n, box, rc, q4, q5, q6, nnb, ws, (size_t)MDPL_SCRATCH_BYTES, stream);
}

mdpl_status mdpl_cna(const double* x, const double* y, const double* z, int64_t n,
                     const double* box, double rc, int32_t max_nb, uint32_t* trip, int32_t* nnb,
                     uint8_t* label, int32_t* max_count, void* ws, size_t bytes, void* stream) {
  if (!trip || !nnb || !label || max_nb < 1 || max_nb > 64) return MDPL_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  Grid g;
  SortBufs sb;
  int32_t *cs, *perm, *skeys;
  double *sx, *sy, *sz;
  NList nl;
  uint32_t* small;
  mdpl_status v = analysis_prep(x, y, z, n, box, rc, max_nb, ws, bytes, st, &g, &sb, &cs, &perm,
                                &sx, &sy, &sz, &skeys, &nl, &small);
  if (v != MDPL_OK) return v;
  HIP_TRY(hipMemsetAsync(small, 0, 64, st));
  HIP_TRY(build_nlist(sx, sy, sz, skeys, cs, n, g, rc * rc, nl, small, (int32_t*)(small + 1), st));
  HIP_TRY(cna_signatures(nl, sx, sy, sz, g, rc * rc, perm, n, trip, nnb, label, max_nb, st));
  if (max_count)
    HIP_TRY(hipMemcpyAsync(max_count, small + 1, 4, hipMemcpyDeviceToDevice, st));
  return MDPL_OK;
}

// ------------------------------------------------------- learned potential
mdpl_status mdpl_desc_fwd(mdpl_sim* s, const double* x, const double* y, const double* z, float* G,
                          float* mom) {
  if (!s || !x || !y || !z || !G || s->tl.half || s->tl.cells) return MDPL_EINVAL;
  if (!s->built) return MDPL_ESTATE;
  HIP_TRY(gather_canonical(x, y, z, s->perm, s->skeys, s->n, s->g, s->sx, s->sy, s->sz, s->st));
  HIP_TRY(desc_forward(s->sx, s->sy, s->sz, s->cell_start, s->g, s->tl, (float)s->p.rc, s->perm, G,
                       mom, s->st));
  return MDPL_OK;
}

mdpl_status mdpl_desc_bwd(mdpl_sim* s, const double* x, const double* y, const double* z,
                          const float* dEdG, const float* mom, float* fx, float* fy,
                          float* fz) {
  if (!s || !x || !y || !z || !dEdG || !mom || !fx || !fy || !fz || s->tl.half || s->tl.cells)
    return MDPL_EINVAL;
  if (!s->built) return MDPL_ESTATE;
  HIP_TRY(gather_canonical(x, y, z, s->perm, s->skeys, s->n, s->g, s->sx, s->sy, s->sz, s->st));
  HIP_TRY(desc_backward(s->sx, s->sy, s->sz, s->cell_start, s->g, s->tl, (float)s->p.rc, s->perm,
                        dEdG, mom, s->n, fx, fy, fz, s->st));
  return MDPL_OK;
}

static bool mlp_ok(const mdpl_mlp_weights* w) {
  return w && w->w1 && w->b1 && w->w2 && w->b2 && w->w3 && w->b3 && w->mu && w->sd &&
         isfinite(w->e_mean) && isfinite(w->e_sd);
}

static MlpArgs mlp_args(const mdpl_mlp_weights* w, const float* G, int64_t n) {
  MlpArgs a;
  a.w1 = w->w1;
  a.b1 = w->b1;
  a.w2 = w->w2;
  a.b2 = w->b2;
  a.w3 = w->w3;
  a.b3 = w->b3;
  a.mu = w->mu;
  a.sd = w->sd;
  a.e_mean = w->e_mean;
  a.e_sd = w->e_sd;
  a.G = G;
  a.index = nullptr;
  a.n = n;
  a.energy = nullptr;
  a.dEdG = nullptr;
  a.target = nullptr;
  a.partial = nullptr;
  a.inv_batch = 0.0f;
  return a;
}

mdpl_status mdpl_mlp_fwd(const mdpl_mlp_weights* w, const float* G, int64_t n, float* energy,
                         float* dEdG, void* stream) {
  if (!mlp_ok(w) || !G || n <= 0 || (!energy && !dEdG)) return MDPL_EINVAL;
  MlpArgs a = mlp_args(w, G, n);
  a.energy = energy;
  a.dEdG = dEdG;
  HIP_TRY(mlp_eval(a, (hipStream_t)stream));
  return MDPL_OK;
}

mdpl_status mdpl_mlp_forces(mdpl_sim* s, const mdpl_mlp_weights* w, const double* x,
                            const double* y, const double* z, float* ws, int64_t ws_floats,
                            float* energy, float* fx, float* fy, float* fz) {
  if (!s || !mlp_ok(w) || !x || !y || !z || !ws || !fx || !fy || !fz || s->tl.half ||
      s->tl.cells)
    return MDPL_EINVAL;
  if (!s->built) return MDPL_ESTATE;
  const int64_t n = s->n;
  if (ws_floats < (int64_t)kMlpRunFloats * n) return MDPL_EWORKSPACE;
  float* G = ws;
  float* mom = G + 24 * n;
  float* e = mom + 50 * n;
  float* dG = e + n;
  HIP_TRY(gather_canonical(x, y, z, s->perm, s->skeys, n, s->g, s->sx, s->sy, s->sz, s->st));
  HIP_TRY(desc_forward(s->sx, s->sy, s->sz, s->cell_start, s->g, s->tl, (float)s->p.rc, s->perm, G,
                       mom, s->st, fx, fy, fz));
  MlpArgs a = mlp_args(w, G, n);
  a.energy = energy ? energy : e;
  a.dEdG = dG;
  HIP_TRY(mlp_eval(a, s->st));
  HIP_TRY(desc_backward(s->sx, s->sy, s->sz, s->cell_start, s->g, s->tl, (float)s->p.rc, s->perm,
                        dG, mom, n, fx, fy, fz, s->st, true));
  return MDPL_OK;
}

mdpl_status mdpl_mlp_train_floats(int64_t batch, int64_t* floats) {
  if (batch <= 0 || !floats) return MDPL_EINVAL;
  *floats = (int64_t)mlp_train_waves(batch) * (kMlpParams + 1);
  return MDPL_OK;
}

mdpl_status mdpl_mlp_train_grad(const mdpl_mlp_weights* w, const float* G, const int32_t* index,
                                int64_t batch, const double* target, float* scratch,
                                int64_t scratch_floats, float* grad, void* stream) {
  if (!mlp_ok(w) || !G || batch <= 0 || !target || !scratch || !grad) return MDPL_EINVAL;
  const int waves = mlp_train_waves(batch);
  if (scratch_floats < (int64_t)waves * (kMlpParams + 1)) return MDPL_EWORKSPACE;
  MlpArgs a = mlp_args(w, G, batch);
  a.index = index;
  a.target = target;
  a.partial = scratch;
  a.inv_batch = 1.0f / (float)batch;
  HIP_TRY(mlp_train_grad(a, (hipStream_t)stream));
  HIP_TRY(mlp_sum_partials(scratch, waves, grad, (hipStream_t)stream));
  return MDPL_OK;
}

mdpl_status mdpl_mlp_standardise(const float* G, const double* e, int64_t n, float* mu,
                                 float* sd, double* e_stats, double* scratch, void* stream) {
  if (!G || !e || n <= 0 || !mu || !sd || !e_stats || !scratch) return MDPL_EINVAL;
  static_assert(MDPL_MLP_STD_SCRATCH >= kStdBlocks * 25 + 50, "standardisation scratch");
  HIP_TRY(mlp_standardise(G, e, n, mu, sd, e_stats, scratch, (hipStream_t)stream));
  return MDPL_OK;
}

mdpl_status mdpl_mlp_bf16(const float* params, uint16_t* w1, uint16_t* w2, uint16_t* w3,
                          void* stream) {
  if (!params || !w1 || !w2 || !w3) return MDPL_EINVAL;
  HIP_TRY(bf16_weights(params, w1, w2, w3, (hipStream_t)stream));
  return MDPL_OK;
}

mdpl_status mdpl_adam_step(float* params, const float* grad, float* m, float* v, float lr,
                           float beta1, float beta2, float eps, int32_t step, uint16_t* w1,
                           uint16_t* w2, uint16_t* w3, void* stream) {
  if (!params || !grad || !m || !v || !w1 || !w2 || !w3 || step < 1 || !(lr > 0.0f)) return MDPL_EINVAL;
  HIP_TRY(adam_step(params, grad, m, v, lr, beta1, beta2, eps, step, w1, w2, w3,
                    (hipStream_t)stream));
  return MDPL_OK;
}

mdpl_status mdpl_mlp_run_floats(int64_t n, int64_t* floats) {
  if (n <= 0 || !floats) return MDPL_EINVAL;
  *floats = (int64_t)kMlpRunFloats * n;
  return MDPL_OK;
}

mdpl_status mdpl_run_mlp(mdpl_sim* s, const mdpl_mlp_weights* w, float* ws, int64_t ws_floats,
                         double* x, double* y, double* z, double* vx, double* vy, double* vz,
                         float* fx, float* fy, float* fz, int32_t* ids, int64_t nsteps,
                         int32_t sample_every, double* thermo, int32_t start) {
  if (!s || !mlp_ok(w) || !ws || !x || !y || !z || !vx || !vy || !vz || !fx || !fy || !fz || !ids)
    return MDPL_EINVAL;
  if (nsteps < 0 || sample_every < 0 || (sample_every > 0 && !thermo)) return MDPL_EINVAL;
  if (s->p.precision != MDPL_FP32 || s->tl.half || s->tl.cells) return MDPL_EINVAL;
  const int64_t n = s->n;
  if (ws_floats < (int64_t)kMlpRunFloats * n) return MDPL_EWORKSPACE;
  float* G = ws;
  float* mom = G + 24 * n;
  float* e = mom + 50 * n;
  float* dG = e + n;
  const float rc = (float)s->p.rc;
  StateArrays user{x, y, z, vx, vy, vz, fx, fy, fz, ids};
  return run_loop(s, user, nsteps, sample_every, thermo, false,
                  [&](const StateArrays& cur, bool en, double* pe_w, int slot, bool,
                      double* const*, double*, double* disp) -> mdpl_status {
                    hipEvent_t e0 = nullptr, e1 = nullptr;
                    if (timed_launch(s, slot)) {
                      HIP_TRY(take_event(s, &e0));
                      HIP_TRY(take_event(s, &e1));
                      HIP_TRY(hipEventRecord(e0, s->st));
                    }
                    HIP_TRY(desc_forward(cur.x, cur.y, cur.z, s->cell_start, s->g, s->tl, rc,
                                         nullptr, G, mom, s->st, (float*)cur.fx, (float*)cur.fy,
                                         (float*)cur.fz));
                    MlpArgs a = mlp_args(w, G, n);
                    a.energy = e;
                    a.dEdG = dG;
                    HIP_TRY(mlp_eval(a, s->st));
                    HIP_TRY(desc_backward(cur.x, cur.y, cur.z, s->cell_start, s->g, s->tl, rc,
                                          nullptr, dG, mom, n, (float*)cur.fx, (float*)cur.fy,
                                          (float*)cur.fz, s->st, true));
                    if (e1) {
                      HIP_TRY(hipEventRecord(e1, s->st));
                      s->tm.ev[slot].push_back(e0);
                      s->tm.ev[slot].push_back(e1);
                    }
                    if (en && pe_w) {  // PE; no virial (zero); the maximum displacement
                      int nb = 0;
                      HIP_TRY(sum_f32(e, n, s->partials, s->st, &nb));
                      RowOut o{};
                      o.dst[0] = pe_w;
                      o.scale[0] = 1.0;
                      o.zdst = pe_w + 1;
                      if (disp) {
                        o.csrc = s->max_disp;
                        o.cdst = disp;
                      }
                      HIP_TRY(reduce_row(s->partials, nb, 1, 1, o, s->st));
                    }
                    return MDPL_OK;
                  },
                  kKindMLP, start);
}

mdpl_status mdpl_force_error(mdpl_sim* s, const float* fx, const float* fy, const float* fz,
                             const double* gx, const double* gy, const double* gz, double* out) {
  if (!s || !fx || !fy || !fz || !gx || !gy || !gz || !out) return MDPL_EINVAL;
  int nb = 0;
  HIP_TRY(force_diff(fx, fy, fz, gx, gy, gz, s->n, s->partials, s->st, &nb));
  HIP_TRY(reduce_partials(s->partials, nb, 2, 2, out, 1.0, s->st));
  return MDPL_OK;
}

mdpl_status mdpl_scale_velocities(double* vx, double* vy, double* vz, int64_t n, double factor,
                                  void* stream) {
  if (!vx || !vy || !vz || n <= 0 || !isfinite(factor)) return MDPL_EINVAL;
  HIP_TRY(scale_velocities(vx, vy, vz, n, factor, (hipStream_t)stream));
  return MDPL_OK;
}

}  // extern "C"
