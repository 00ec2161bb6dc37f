// Internal declarations shared by the translation units of libmdpl.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mdpl.h"
#include "device_util.h"

namespace mdpl {

constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;                       // keys per thread per tile
constexpr int kSortTile = kSortThreads * kSortItems; // keys per tile
constexpr int kReduceThreads = 256;                  // block size of reducing kernels
constexpr int kMaxCycle = 4096;                      // largest reuse_every

inline int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Cell grid: nc[k] = floor(L_k / (r (1 + 1e-10))) cells of side L_k / nc[k]
// per axis, grouped into bricks of B[0] x B[1] x B[2] cells (the last brick
// along an axis may be partial).  Cell keys are brick-major:
//   key = brick * V + (lz * B[1] + ly) * B[0] + lx,
//   brick = (bz * nb[1] + by) * nb[0] + bx,  V = B[0] B[1] B[2],
// so that sorting particles by key makes every brick a contiguous range.
// With B = (1,1,1) the key is the plain x-fastest cell index.
struct Grid {
  int nc[3];
  int B[3];
  int nb[3];
  int V;
  int nbricks;
  int nkeys;  // nbricks * V
  double inv_side[3];
  double side[3];  // box / nc, the cell edge
  double box[3];
  // tile kernels: brick of each of their norder workgroups (device, nbricks
  // for padding); null: the order of brick_of_block
  const int32_t* order;
  int norder;
};

// Returns MDPL_EBOX if fewer than 3 cells fit along some axis.
mdpl_status make_grid(const double box[3], double r, const int brick[3], Grid* g);

__host__ __device__ inline int cell_key(const Grid& g, int cx, int cy, int cz) {
  const int bx = cx / g.B[0], by = cy / g.B[1], bz = cz / g.B[2];
  const int lx = cx - bx * g.B[0], ly = cy - by * g.B[1], lz = cz - bz * g.B[2];
  return ((bz * g.nb[1] + by) * g.nb[0] + bx) * g.V + (lz * g.B[1] + ly) * g.B[0] + lx;
}

// Radix-sort scratch for n keys.
struct SortBufs {
  int32_t* keys[2];
  int32_t* vals[2];
  int32_t* hist;      // kRadixBins * ntiles, then its block sums
  int32_t* blocksums; // scan scratch
  int64_t n;
  int ntiles;
};
size_t sort_bytes(int64_t n);
void sort_carve(char*& p, int64_t n, SortBufs* s);

// Sort particles by cell: keys computed from (folded) positions, values =
// particle index.  On return keys_out/vals_out point at the sorted arrays
// (one of the two ping-pong buffers) and cell_start[0..ncells] is filled.
hipError_t bin_particles(const double* x, const double* y, const double* z, int64_t n,
                         const Grid& g, SortBufs& s, int32_t* cell_start, int32_t** keys_out,
                         int32_t** vals_out, hipStream_t st, int32_t* xlow = nullptr);

// Exclusive prefix sum of n int32 values into out (may alias in).  Uses
// blocksums scratch of at least div_up(n, 1024) + 1 entries.  Also writes
// the total to out[n] if write_total.
hipError_t exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* blocksums,
                          bool write_total, hipStream_t st);

// Gathers: dst[k] = src[idx[k]] for double / float / int arrays.
hipError_t gather_positions(const double* x, const double* y, const double* z, const int32_t* idx,
                            int64_t n, double* ox, double* oy, double* oz, const double* box,
                            bool fold, hipStream_t st);

// Like gather_positions, but each position is moved to the periodic image
// nearest the centre of its cell in the sorted keys skeys.
hipError_t gather_canonical(const double* x, const double* y, const double* z, const int32_t* idx,
                            const int32_t* skeys, int64_t n, const Grid& g, double* ox, double* oy,
                            double* oz, hipStream_t st);

struct StateArrays {
  double *x, *y, *z, *vx, *vy, *vz;
  void *fx, *fy, *fz;
  int32_t* ids;
};
// dst[s] = src[idx[s]] for all ten arrays, positions folded into the box;
// xb/yb/zb (nullable) receive a copy of the folded positions; bound
// (nullable) is set to zero (a new list: nothing has moved since).
hipError_t reorder_state(const StateArrays& src, const int32_t* idx, int64_t n, int fbytes,
                         const double* box, StateArrays& dst, double* xb, double* yb, double* zb,
                         double* bound, hipStream_t st);

// dst[a] = src[a] for each of the ten arrays whose pointers differ (one launch).
hipError_t copy_state(const StateArrays& src, const StateArrays& dst, int64_t n, int fbytes,
                      hipStream_t st);

// Neighbour list (ELL) of the analysis passes: row-major nbr[i * max_nb + m]
// of sorted-slot indices; cnt[i] is the true count (may exceed max_nb).
// Requires a grid with B = (1,1,1).
struct NList {
  int32_t* nbr;
  int32_t* cnt;
  int64_t stride;
  int max_nb;
  int layout;
};
hipError_t build_nlist(const double* sx, const double* sy, const double* sz,
                       const int32_t* skeys, const int32_t* cell_start, int64_t n, const Grid& g,
                       double r2, NList nl, uint32_t* flags, int32_t* maxcount, hipStream_t st);

// Tiled neighbour list of the LJ path.  One workgroup per brick stages the
// positions of the brick's (B+2)^3-cell neighbourhood (its "tile") in LDS;
// an entry is the neighbour's tile slot as a byte offset (below), 16 bits,
// packed four to a 64-bit word, the words column-major: entry m of slot s
// is 16-bit lane (m & 3) of nbr[(m >> 2) * stride + s].  The last word of a
// list is padded with the offset of kTileDummy, a tile slot that holds a
// position far outside the box.
constexpr int kTileMax = 3072;              // tile slots (LDS)
constexpr int kBrickMax = 1024;             // particles of one brick the list builder counts
constexpr int kTileDummy = kTileMax - 1;    // padding slot
constexpr int kTileCap = kTileMax - 1;      // particles a tile can hold
constexpr int kTileCells = 125;             // B <= 3 per axis
constexpr int kTileMaxHalf = 2144;          // tile slots of a half-list tile (LDS)
// A list entry is the partner's tile slot u as a byte offset: u << 2 in full
// lists (its offset in the 4-byte arrays of the FP32 force tile; the FP64
// kernels scale it), u << 3 in half lists (8-byte arrays).
constexpr int kFullShift = 2;
constexpr int kHalfShift = 3;
// Per-brick tile tables of the full lists (prefix, src, code of tile.h),
// written by the list build for the force pass, which then need not derive
// them every step: kTabInts ints per brick.
constexpr int kTabInts = (kTileCells + 1) + 2 * kTileCells;
struct TileList {
  uint64_t* nbr;
  int32_t* cnt;     // clamped to max_nb
  int32_t* tab;     // nbricks * kTabInts (full lists; null: not kept)
  int64_t stride;   // words per group row (>= n)
  int max_nb;       // multiple of 4
  int threads;      // workgroup size of the tile kernels
  int half;         // 1: each pair once (Newton's third law), tiles of kTileMaxHalf slots
  int cells;        // 1: no list; the pair loop scans the cell stencil (nbr and cnt unused)
  // per cell key, its particles in the lower half of the cell along x (they
  // come first in the cell); null: the list build scans whole stencil rows
  int32_t* xlow;
};
hipError_t build_tile_nlist(const double* x, const double* y, const double* z,
                            const int32_t* skeys, const int32_t* cell_start, const Grid& g,
                            double r2, TileList tl, uint32_t* flags, int32_t* maxcount,
                            hipStream_t st);
hipError_t export_tile_pairs(const TileList& tl, const int32_t* cell_start, const Grid& g,
                             const int32_t* perm, const int32_t* offsets, int32_t* i_out,
                             int32_t* j_out, int64_t cap, hipStream_t st);

// Lennard-Jones pair constants.
struct LJConst {
  double rc2, eps, sigma2, shift_v;  // shift_v added to every pair energy
  double box[3], half[3], inv_box[3];
};

// Rebuild rule of Eq. extended_cutoff: every kernel that drifts the
// positions (the fused force pass or k_vv) stores the largest |v|^2 of each
// workgroup; workgroup 0 of the next drifting launch, when that launch has
// ended, reduces them, adds dt * max|v| to bound (the sum over the steps
// since the last build, an upper bound of every particle's displacement) and
// publishes {bound, max|v|} with the step index in a ring of host-visible
// records, so that the host can decide on a rebuild without waiting for the
// stream.  No atomics and no device-scope fences are needed (the launch
// boundary orders the maxima before their reduction).  The host publishes a
// pending record with k_publish when it must decide at once; the rebuild
// (k_reorder) sets bound back to zero and drops the pending record.
struct KickRecord {
  int64_t stamp;  // global step index of the positions the drift produced (-1: empty)
  double bound;   // sum of dt * max|v| since the last build, this step included
  double vmax;    // largest speed of the step
  double pad;
};
constexpr int kRing = 64;  // records kept (indexed by stamp mod kRing)
struct KickTrack {
  double* part[2];    // device: per-workgroup largest |v|^2 of the last two drifting launches
  double* bound;      // device
  KickRecord* ring;   // host-visible records (device address); null: no tracking
  int64_t step;       // global step index of the positions this launch produces
  int64_t pub_step;   // step index of the record to publish first
  int pub_n;          // workgroups of the launch that produced it (0: none pending)
  int cur;            // part[cur] takes this launch's maxima; part[cur ^ 1] holds the pending ones
  double dt;
};
// Thread 0 of every workgroup of a drifting launch: the workgroup's largest
// |v|^2 (0 without particles; a non-finite value counts as infinite).
__device__ inline void kick_store(const KickTrack& kt, double m2) {
  if (!kt.ring) return;
  kt.part[kt.cur][blockIdx.x] = m2 >= 0.0 ? m2 : __builtin_huge_val();
}
// Every thread of workgroup 0 of a drifting launch, before its other work
// (no-op elsewhere): the pending record.  sh: one double per wave.
__device__ inline void kick_publish(const KickTrack& kt, double* sh) {
  if (!kt.ring || kt.pub_n <= 0 || blockIdx.x != 0) return;
  const double* p = kt.part[kt.cur ^ 1];
  double m = 0.0;
  for (int i = threadIdx.x; i < kt.pub_n; i += blockDim.x) m = p[i] > m ? p[i] : m;
  m = wave_max_nonneg(m);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 1; w < nw; ++w) m = sh[w] > m ? sh[w] : m;
    const double vmax = sqrt(m);
    const double b = *kt.bound + kt.dt * vmax;
    *kt.bound = b;
    KickRecord* r = kt.ring + (kt.pub_step & (kRing - 1));
    r->bound = b;
    r->vmax = vmax;
    __threadfence_system();
    __hip_atomic_store(&r->stamp, kt.pub_step, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  __syncthreads();
}
// The pending record alone (one workgroup).
hipError_t publish_record(const KickTrack& kt, hipStream_t st);

struct ForceOut {
  void *fx, *fy, *fz;     // force arrays (float or double)
  const int32_t* scatter; // nullable: slot s writes to scatter[s]
  double* e_atom;         // nullable (scattered like forces)
  double* partials;       // per-block {pe, w} ({pe, w, 2 ke} when fused) when energy is on
  double scale;           // multiplies the stored force (backward: -grad)
  const double* scale_dev;// nullable: device scalar multiplying the stored force
  // Fused velocity-Verlet (run loop only; forces are then not stored):
  // v += h F ; [ke] ; v += h F ; r_new = r + dt v, exactly as vv_step mode 1.
  bool fuse;
  double *vx, *vy, *vz;   // velocities, updated in place
  double *nx, *ny, *nz;   // new positions (a different buffer from x, y, z)
  double h, dt;
  uint32_t* flags;        // MDPL_FLAG_NONFINITE on a non-finite velocity; tile overflow (no list)
  KickTrack track;        // fused drift: the step's largest speed (rebuild rule)
};
// Partials are written per brick (nblocks_out = number of bricks).
hipError_t lj_force(const double* x, const double* y, const double* z, const int32_t* cell_start,
                    const Grid& g, const TileList& tl, const LJConst& c, int precision, bool energy,
                    const ForceOut& out, int64_t n, hipStream_t st, int* nblocks_out);
// the same with half lists (outputs cleared, then summed with atomics) and
// with no list (the cell stencil)
hipError_t lj_force_half(const double* x, const double* y, const double* z,
                         const int32_t* cell_start, const Grid& g, const TileList& tl,
                         const LJConst& c, int precision, bool energy, const ForceOut& out,
                         int64_t n, hipStream_t st);
hipError_t lj_force_cells(const double* x, const double* y, const double* z,
                          const int32_t* cell_start, const Grid& g, const LJConst& c,
                          int precision, bool energy, const ForceOut& out, hipStream_t st);

// Velocity Verlet particle loops on the sorted state (INC on v and r).
// Andersen collisions (Sec. 5.2) applied by vv_step right after the kick
// that completes a step (modes 1 and 2), after the KE sample: particle s
// collides with probability p and takes sd * (n1, n2, n3), the draws from
// Philox4x64-10 with key (seed, 0) and counter (step, ids[s], block, 0).
struct Andersen {
  const int32_t* ids;  // particle ids of the slots: the random streams follow the particles
  double p;            // collision probability per particle and step (nu dt); 0: none
  double sd;           // sqrt(T / m)
  uint64_t seed;
  int64_t step;        // global index of the step that the kick completes
};
//   mode 0: v += h F ; r' = r + dt v                          (first step)
//   mode 1: v += h F ; [KE] ; [collide] ; v += h F ; r' = r + dt v   (fused end+start)
//   mode 2: v += h F ; [KE] ; [collide]                       (final half kick)
//   mode 3: KE only
// The drifted positions r' go to nx, ny, nz (a buffer other than x, y, z, so
// that the positions of the last force pass survive the step); modes 0 and
// 1 report the step's largest speed to track (nullable).
hipError_t vv_step(const double* x, const double* y, const double* z, double* nx, double* ny,
                   double* nz, double* vx, double* vy, double* vz, const void* fx, const void* fy,
                   const void* fz, int precision, int64_t n, double h, double dt, int mode, bool ke,
                   double* ke_partials, uint32_t* flags, hipStream_t st, int* nblocks_out,
                   const Andersen* th = nullptr, const KickTrack* track = nullptr);

// out[0] = sum of partials[k * stride + comp] over k, fixed order, one block.
hipError_t reduce_partials(const double* partials, int nblocks, int stride, int ncomp,
                           double* out, double scale, hipStream_t st);

// Destinations of reduce_row: dst[c] = scale[c] * (sum of component c), each
// skipped if null; then *cdst = *csrc and *zdst = 0 where given.
struct RowOut {
  double* dst[3];
  double scale[3];
  const double* csrc;
  double* cdst;
  double* zdst;
};
// Up to three components (the sums of reduce_partials, same order) and the
// copy/zero of RowOut in one launch.
hipError_t reduce_row(const double* partials, int nblocks, int stride, int ncomp, const RowOut& o,
                      hipStream_t st);

// Per-block maxima of |r - r_build|^2 into partials.
hipError_t disp_partials(const double* x, const double* y, const double* z, const double* xb,
                         const double* yb, const double* zb, int64_t n, double* partials,
                         hipStream_t st, int* nblocks_out);

// d = sqrt(max partials); *max_disp = max(*max_disp, d); flags |= SKIN if d >= half_skin.
hipError_t skin_check(const double* partials, int nblocks, double half_skin, double* max_disp,
                      uint32_t* flags, hipStream_t st);

// Analysis kernels on sorted positions.
hipError_t boa_q(const double* sx, const double* sy, const double* sz, const int32_t* skeys,
                 const int32_t* cell_start, const int32_t* perm, int64_t n, const Grid& g,
                 double rc2, float* q4, float* q5, float* q6, int32_t* nnb, hipStream_t st);

// CNA of every particle from its complete list (adjacency among its
// neighbours from the exact bond test on the sorted positions sx, sy, sz).
hipError_t cna_signatures(const NList& nl, const double* sx, const double* sy, const double* sz,
                          const Grid& g, double rc2, const int32_t* perm, int64_t n,
                          uint32_t* trip, int32_t* nnb, uint8_t* label, int max_out,
                          hipStream_t st);


// Learned potential: descriptors (desc.hip) and dense layers (mlp.hip).
// desc_forward also clears fx, fy, fz (caller order) when they are given, so
// that a following desc_backward with zeroed = true needs no clearing launch.
hipError_t desc_forward(const double* x, const double* y, const double* z,
                        const int32_t* cell_start, const Grid& g, const TileList& tl, float rc,
                        const int32_t* perm, float* G, float* mom, hipStream_t st,
                        float* fx = nullptr, float* fy = nullptr, float* fz = nullptr);
hipError_t desc_backward(const double* x, const double* y, const double* z,
                         const int32_t* cell_start, const Grid& g, const TileList& tl, float rc,
                         const int32_t* perm, const float* dEdG, const float* mom, int64_t n,
                         float* fx, float* fy, float* fz, hipStream_t st, bool zeroed = false);

struct MlpArgs;
hipError_t mlp_eval(const MlpArgs& a, hipStream_t st);
hipError_t mlp_train_grad(const MlpArgs& a, hipStream_t st);
int mlp_train_waves(int64_t n);
hipError_t mlp_sum_partials(const float* partial, int nwaves, float* out, hipStream_t st);
hipError_t adam_step(float* p, const float* g, float* m, float* v, float lr, float b1, float b2,
                     float eps, int t, unsigned short* w1, unsigned short* w2, unsigned short* w3,
                     hipStream_t st);
// BF16 copies of the weight matrices (w1, w2, w3) of packed FP32 parameters.
hipError_t bf16_weights(const float* p, unsigned short* w1, unsigned short* w2, unsigned short* w3,
                        hipStream_t st);
// Feature means mu and spreads sd (24 floats each), energy mean and spread
// (e_stats, 2 doubles) of n training rows; scratch: kStdBlocks * 25 + 50 doubles.
constexpr int kStdBlocks = 256;
hipError_t mlp_standardise(const float* G, const double* e, int64_t n, float* mu, float* sd,
                           double* e_stats, double* scratch, hipStream_t st);
hipError_t scale_velocities(double* vx, double* vy, double* vz, int64_t n, double factor,
                            hipStream_t st);
// FP64 block partials of a float array, and of (|f - g|^2, |g|^2) per particle.
hipError_t sum_f32(const float* v, int64_t n, double* partials, hipStream_t st, int* nblocks_out);
hipError_t force_diff(const float* fx, const float* fy, const float* fz, const double* gx,
                      const double* gy, const double* gz, int64_t n, double* partials,
                      hipStream_t st, int* nblocks_out);

}  // namespace mdpl
