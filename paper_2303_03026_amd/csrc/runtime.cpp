// Host runtime of the C ABI declared in include/amrvac.h.
//
// A context owns a pool of block places (the caller's slots hold the data)
// and a set of jobs, each a 2:1-nested leaf-block hierarchy occupying a
// contiguous run of pool places.  For every job the runtime validates the
// hierarchy, builds face-neighbour links and ghost-task lists, and keeps
// per-block tables (level, job, spacing, links) and per-job CFL geometry on
// the device.  A single-job context (amrvac_init_blocks) is one job over
// the whole pool; a batch context (amrvac_batch_create) admits and retires
// jobs between steps and advances all active jobs together.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <unordered_set>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/amrvac.h"
#include "kernels.h"

using namespace amrvac;

namespace {

struct KeyL {
  int l;
  long i, j, k;
  bool operator<(const KeyL& o) const { return std::tie(l, i, j, k) < std::tie(o.l, o.i, o.j, o.k); }
  bool operator==(const KeyL& o) const { return l == o.l && i == o.i && j == o.j && k == o.k; }
};

// Hash of a block key (splitmix64 finaliser over the packed coordinates):
// the block tables and the regrid planner look blocks up by key hundreds of
// thousands of times per call.
struct KeyHash {
  size_t operator()(const KeyL& q) const noexcept {
    unsigned long long h = (unsigned long long)q.l;
    h = h * 0x100000001B3ull ^ (unsigned long long)q.i;
    h = h * 0x100000001B3ull ^ (unsigned long long)q.j;
    h = h * 0x100000001B3ull ^ (unsigned long long)q.k;
    h ^= h >> 30;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 27;
    h *= 0x94D049BB133111EBull;
    h ^= h >> 31;
    return (size_t)h;
  }
};
using KeyMap = std::unordered_map<KeyL, int, KeyHash>;
using KeySet = std::unordered_set<KeyL, KeyHash>;

// Validated tables of one job's hierarchy (pool ids already offset).
struct JobBuild {
  std::string err;
  int finest = 1;
  std::vector<int> level, link, pos, wrap, order_local;
  std::vector<double> invdx;
  std::vector<int> tfill, tfused, tprol, trefl;  // (pool block, face) pairs
  double geom[4] = {0, 0, 0, 0};  // sum_d 1/dx_d (finest), min_d dx_d (finest), cfl, glm_alpha
};

// Per-job host record.
struct JobRec {
  bool used = false;
  int first = 0;
  int nb = 0;
  int steps_left = 0;
  int steps_done = 0;
  JobBuild t;
};

int check_desc(const amrvac_grid_desc* g, std::string* why) {
  if (!g) { *why = "null descriptor"; return AMRVAC_E_ARG; }
  if (g->ndim != 2 && g->ndim != 3) { *why = "ndim must be 2 or 3"; return AMRVAC_E_ARG; }
  if (g->nghost != 2 && g->nghost != 3) { *why = "nghost must be 2 or 3"; return AMRVAC_E_ARG; }
  if (g->block_nx < 4 || g->block_nx > 16 || (g->block_nx & 1)) { *why = "block_nx must be even, 4..16"; return AMRVAC_E_ARG; }
  // a coarse ghost layer of depth nghost is restricted from 2 nghost fine
  // cells, which must lie inside the fine neighbour
  if (2 * g->nghost > g->block_nx) { *why = "block_nx must be at least 2 nghost"; return AMRVAC_E_ARG; }
  if (g->precision != AMRVAC_FP64 && g->precision != AMRVAC_FP32_MIXED) { *why = "bad precision"; return AMRVAC_E_ARG; }
  for (int d = 0; d < g->ndim; ++d) {
    if (g->base_blocks[d] < 1) { *why = "base_blocks must be >= 1"; return AMRVAC_E_ARG; }
    if (!(g->xmax[d] > g->xmin[d])) { *why = "xmax must exceed xmin"; return AMRVAC_E_ARG; }
    for (int s = 0; s < 2; ++s) {
      const int bc = s ? g->bc_hi[d] : g->bc_lo[d];
      if (bc < 0 || bc > 3) { *why = "bad boundary kind"; return AMRVAC_E_ARG; }
    }
    if ((g->bc_lo[d] == AMRVAC_BC_PERIODIC) != (g->bc_hi[d] == AMRVAC_BC_PERIODIC)) {
      *why = "periodic boundaries must be periodic on both sides";
      return AMRVAC_E_ARG;
    }
  }
  if (!(g->gamma > 1.0) || !(g->cfl > 0.0) || !(g->glm_alpha >= 0.0)) { *why = "bad gamma/cfl/glm_alpha"; return AMRVAC_E_ARG; }
  if (g->limiter < AMRVAC_LIM_VANLEER || g->limiter > AMRVAC_LIM_WENOZP5) { *why = "bad limiter"; return AMRVAC_E_ARG; }
  if (g->limiter >= AMRVAC_LIM_WENO5 && g->nghost != 3) {
    *why = "the five-cell reconstructions (weno5, wenoz5, mp5, wenozp5) need nghost = 3";
    return AMRVAC_E_ARG;
  }
  if (g->flux < AMRVAC_FLUX_HLL || g->flux > AMRVAC_FLUX_HLLC) { *why = "bad flux scheme"; return AMRVAC_E_ARG; }
  if (g->precision == AMRVAC_FP32_MIXED && g->block_nx != 16) {
    *why = "FP32-mixed storage runs on the fused path, which needs block_nx = 16";
    return AMRVAC_E_ARG;
  }
  return AMRVAC_OK;
}

// bytes before the first block of a slot (FP64: interior rows start at
// x = 2 doubles = 16 B into a padded row; the lead moves them onto 32 B
// memory sectors, which every pitch of the FP64 layout is a multiple of)
long slot_lead(int precision) { return precision == AMRVAC_FP64 ? AMRVAC_SLOT_LEAD_FP64 : 0; }

long long slot_bytes_of(const amrvac_grid_desc* g, long nb) {
  const long pn = g->block_nx + 2 * g->nghost;
  const long pc = pn * pn * (g->ndim == 3 ? pn : 1);
  const long per = g->precision == AMRVAC_FP64 ? 72 : 40;
  return (long long)nb * pc * per + slot_lead(g->precision);
}

// Leaf / refined-slot lookup for build_job.  Per level a dense array over
// the level's block slots (-1 empty, -2 refined, else the leaf's index) when
// all levels together have at most kDenseSlots slots, else hash maps; block
// tables are built for every init, batch admission and regrid, so this is
// the hot part of validating a hierarchy.
class BlockLookup {
 public:
  static constexpr long kDenseSlots = 1L << 24;
  BlockLookup(int ndim, const int* base, int finest, int nb) {
    long total = 0;
    for (int l = 1; l <= finest; ++l) {
      long n = 1;
      for (int d = 0; d < 3; ++d) n *= d < ndim ? ((long)base[d] << (l - 1)) : 1;
      total += n;
      if (total > kDenseSlots) break;
    }
    dense_ = total <= kDenseSlots;
    if (dense_) {
      off_.assign(finest + 2, 0);
      for (int l = 1; l <= finest; ++l) {
        for (int d = 0; d < 3; ++d) dim_[l][d] = d < ndim ? ((long)base[d] << (l - 1)) : 1;
        off_[l + 1] = off_[l] + dim_[l][0] * dim_[l][1] * dim_[l][2];
      }
      cells_.assign(off_[finest + 1], -1);
      finest_ = finest;
    } else {
      leaf_.reserve((size_t)nb * 2);
      refined_.reserve((size_t)nb);
    }
  }
  // false if the slot already holds a leaf; a leaf on a refined slot (or the
  // reverse) is recorded as an overlap
  bool add_leaf(const KeyL& k, int id) {
    if (!dense_) {
      if (!leaf_.emplace(k, id).second) return false;
      if (refined_.count(k)) overlap_ = true;
      return true;
    }
    int& c = cells_[index(k)];
    if (c >= 0) return false;
    if (c == -2) overlap_ = true;
    c = id;
    return true;
  }
  void add_refined(const KeyL& k) {
    if (!dense_) {
      refined_.insert(k);
      if (leaf_.count(k)) overlap_ = true;
      return;
    }
    int& c = cells_[index(k)];
    if (c >= 0) overlap_ = true;
    else c = -2;
  }
  bool overlap() const { return overlap_; }
  // the leaf's index at slot k of level k.l, or -1
  int leaf(const KeyL& k) const {
    if (!dense_) {
      auto it = leaf_.find(k);
      return it == leaf_.end() ? -1 : it->second;
    }
    if (k.l < 1 || k.l > finest_) return -1;
    const int c = cells_[index(k)];
    return c >= 0 ? c : -1;
  }
  bool refined(const KeyL& k) const {
    if (!dense_) return refined_.count(k) != 0;
    if (k.l < 1 || k.l > finest_) return false;
    return cells_[index(k)] == -2;
  }

 private:
  long index(const KeyL& k) const { return off_[k.l] + (k.k * dim_[k.l][1] + k.j) * dim_[k.l][0] + k.i; }
  bool dense_ = false, overlap_ = false;
  int finest_ = 0;
  long dim_[MAXLEV + 2][3] = {};
  std::vector<long> off_;
  std::vector<int> cells_;
  KeyMap leaf_;
  KeySet refined_;
};

// Validate a job's leaf blocks and build its tables with pool ids starting
// at `first`.  Host only: no device call.
int build_job(const amrvac_grid_desc* g, int nb, const int* level, const int* ijk, int first, JobBuild* out) {
  JobBuild& J = *out;
  const int ndim = g->ndim, nx = g->block_nx;
  for (int b = 0; b < nb; ++b) {
    const int l = level[b];
    if (l < 1 || l > MAXLEV) { J.err = "level out of range 1..12"; return AMRVAC_E_ARG; }
    const long p[3] = {ijk[3 * b], ijk[3 * b + 1], ndim == 3 ? ijk[3 * b + 2] : 0};
    for (int d = 0; d < ndim; ++d)
      if (p[d] < 0 || p[d] >= ((long)g->base_blocks[d] << (l - 1))) { J.err = "block outside the domain"; return AMRVAC_E_ARG; }
    J.finest = std::max(J.finest, l);
  }
  BlockLookup look(ndim, g->base_blocks, J.finest, nb);
  double vol = 0.0;
  for (int b = 0; b < nb; ++b) {
    const int l = level[b];
    long p[3] = {ijk[3 * b], ijk[3 * b + 1], ndim == 3 ? ijk[3 * b + 2] : 0};
    if (!look.add_leaf(KeyL{l, p[0], p[1], p[2]}, b)) { J.err = "duplicate block"; return AMRVAC_E_ARG; }
    vol += std::ldexp(1.0, -ndim * (l - 1));
    for (int m = l - 1; m >= 1; --m) {
      for (int d = 0; d < 3; ++d) p[d] >>= 1;
      look.add_refined(KeyL{m, p[0], p[1], p[2]});
    }
  }
  if (look.overlap()) { J.err = "blocks overlap (a leaf is also refined)"; return AMRVAC_E_ARG; }
  const double nbase = (double)g->base_blocks[0] * g->base_blocks[1] * (ndim == 3 ? g->base_blocks[2] : 1);
  if (std::fabs(vol - nbase) > 1e-9 * nbase) { J.err = "blocks do not tile the domain"; return AMRVAC_E_ARG; }

  auto nblk = [&](int l, int d) -> long { return d < ndim ? ((long)g->base_blocks[d] << (l - 1)) : 1; };
  auto periodic = [&](int d) { return g->bc_lo[d] == AMRVAC_BC_PERIODIC; };
  // 2:1 nesting over faces, edges and corners: every slot next to a leaf of
  // level l is a leaf, refined into leaves, or inside a leaf of level l-1.
  for (int b = 0; b < nb; ++b) {
    const int l = level[b];
    const long p[3] = {ijk[3 * b], ijk[3 * b + 1], ndim == 3 ? ijk[3 * b + 2] : 0};
    for (int oz = (ndim == 3 ? -1 : 0); oz <= (ndim == 3 ? 1 : 0); ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          long q[3] = {p[0] + ox, p[1] + oy, p[2] + oz};
          bool skip = false;
          for (int d = 0; d < ndim; ++d)
            if (q[d] < 0 || q[d] >= nblk(l, d)) {
              if (periodic(d)) q[d] = (q[d] + nblk(l, d)) % nblk(l, d);
              else skip = true;
            }
          if (skip) continue;
          const KeyL k{l, q[0], q[1], q[2]};
          if (look.leaf(k) >= 0) continue;
          if (look.refined(k)) {
            const long off[3] = {ox, oy, oz};
            for (int cz = 0; cz < (ndim == 3 ? 2 : 1); ++cz)
              for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx) {
                  const long cc[3] = {cx, cy, cz};
                  bool adjacent = true;
                  for (int d = 0; d < ndim; ++d) {
                    if (off[d] == 1 && cc[d] != 0) adjacent = false;
                    if (off[d] == -1 && cc[d] != 1) adjacent = false;
                  }
                  if (!adjacent) continue;
                  const KeyL ck{l + 1, 2 * q[0] + cx, 2 * q[1] + cy, ndim == 3 ? 2 * q[2] + cz : 0};
                  if (look.leaf(ck) < 0) { J.err = "hierarchy is not 2:1 nested (finer by two)"; return AMRVAC_E_ARG; }
                }
            continue;
          }
          if (l >= 2 && look.leaf(KeyL{l - 1, q[0] >> 1, q[1] >> 1, ndim == 3 ? q[2] >> 1 : 0}) >= 0) continue;
          J.err = "hierarchy is not 2:1 nested (coarser by two)";
          return AMRVAC_E_ARG;
        }
  }

  J.level.assign(nb, 0);
  J.pos.assign((size_t)nb * 3, 0);
  J.wrap.assign((size_t)nb * 3, 1);
  J.invdx.assign((size_t)nb * 3, 1.0);
  J.link.assign((size_t)nb * 6 * LINK_INTS, -1);
  for (int b = 0; b < nb; ++b) {
    const int l = level[b];
    J.level[b] = l;
    const long p[3] = {ijk[3 * b], ijk[3 * b + 1], ndim == 3 ? ijk[3 * b + 2] : 0};
    for (int d = 0; d < 3; ++d) {
      J.pos[3 * b + d] = (int)p[d];
      J.wrap[3 * b + d] = (int)(nblk(l, d) * nx);
      J.invdx[3 * b + d] = d < ndim ? 1.0 / ((g->xmax[d] - g->xmin[d]) / (double)(nblk(l, d) * nx)) : 1.0;
    }
    for (int d = 0; d < ndim; ++d)
      for (int side = 0; side < 2; ++side) {
        int* Lk = &J.link[((size_t)b * 6 + d * 2 + side) * LINK_INTS];
        long q[3] = {p[0], p[1], p[2]};
        q[d] += side ? 1 : -1;
        if (q[d] < 0 || q[d] >= nblk(l, d)) {
          if (!periodic(d)) {
            Lk[0] = LINK_PHYS;
            Lk[1] = side ? g->bc_hi[d] : g->bc_lo[d];
            J.tfill.push_back(first + b);
            J.tfill.push_back(d * 2 + side);
            continue;
          }
          q[d] = (q[d] + nblk(l, d)) % nblk(l, d);
        }
        const int same = look.leaf(KeyL{l, q[0], q[1], q[2]});
        if (same >= 0) {
          Lk[0] = LINK_SAME;
          Lk[1] = first + same;
          J.tfill.push_back(first + b);
          J.tfill.push_back(d * 2 + side);
          continue;
        }
        if (look.refined(KeyL{l, q[0], q[1], q[2]})) {
          Lk[0] = LINK_FINE;
          const int ta = d == 0 ? 1 : 0, tb = d == 2 ? 1 : 2;
          for (int ob = 0; ob < (ndim == 3 ? 2 : 1); ++ob)
            for (int oa = 0; oa < 2; ++oa) {
              long cq[3] = {2 * q[0], 2 * q[1], ndim == 3 ? 2 * q[2] : 0};
              cq[d] += side ? 0 : 1;
              cq[ta] += oa;
              if (ndim == 3) cq[tb] += ob;
              const int ci = look.leaf(KeyL{l + 1, cq[0], cq[1], cq[2]});
              if (ci < 0) { J.err = "fine neighbour is not a leaf"; return AMRVAC_E_ARG; }
              Lk[1 + ob * 2 + oa] = first + ci;
            }
          J.tfill.push_back(first + b);
          J.tfill.push_back(d * 2 + side);
          J.trefl.push_back(first + b);
          J.trefl.push_back(d * 2 + side);
          continue;
        }
        const int pi = l >= 2 ? look.leaf(KeyL{l - 1, q[0] >> 1, q[1] >> 1, ndim == 3 ? q[2] >> 1 : 0}) : -1;
        if (pi < 0) { J.err = "face neighbour not found (hierarchy not 2:1 nested)"; return AMRVAC_E_ARG; }
        Lk[0] = LINK_COARSE;
        Lk[1] = first + pi;
        Lk[2] = l;
        J.tprol.push_back(first + b);
        J.tprol.push_back(d * 2 + side);
      }
  }
  if (!g->reflux) J.trefl.clear();
  // The fused stage and the prolongation read same-level neighbours in place;
  // the fused path fills ghosts only on faces towards finer leaves and
  // physical boundaries (then prolongs the faces towards coarser ones).
  for (size_t q = 0; q < J.tfill.size(); q += 2) {
    const int lb = J.tfill[q] - first, face = J.tfill[q + 1];
    if (J.link[((size_t)lb * 6 + face) * LINK_INTS] != LINK_SAME) {
      J.tfused.push_back(J.tfill[q]);
      J.tfused.push_back(face);
    }
  }
  // Morton order on the finest level's block grid
  std::vector<std::pair<unsigned long long, int>> keyed(nb);
  for (int b = 0; b < nb; ++b) {
    const int sft = J.finest - J.level[b];
    unsigned long long key = 0;
    const unsigned long long q0 = (unsigned long long)J.pos[3 * b] << sft;
    const unsigned long long q1 = (unsigned long long)J.pos[3 * b + 1] << sft;
    const unsigned long long q2 = (unsigned long long)J.pos[3 * b + 2] << sft;
    for (int bit = 0; bit < 20; ++bit) {
      key |= ((q0 >> bit) & 1ull) << (3 * bit);
      key |= ((q1 >> bit) & 1ull) << (3 * bit + 1);
      key |= ((q2 >> bit) & 1ull) << (3 * bit + 2);
    }
    keyed[b] = {key, b};
  }
  std::sort(keyed.begin(), keyed.end());
  J.order_local.resize(nb);
  for (int b = 0; b < nb; ++b) J.order_local[b] = first + keyed[b].second;
  // CFL geometry on the finest level
  double sum_inv = 0.0, min_dx = 0.0;
  for (int d = 0; d < ndim; ++d) {
    const double dx = (g->xmax[d] - g->xmin[d]) / (double)(nblk(J.finest, d) * nx);
    sum_inv += 1.0 / dx;
    min_dx = d == 0 ? dx : std::min(min_dx, dx);
  }
  J.geom[0] = sum_inv;
  J.geom[1] = min_dx;
  J.geom[2] = g->cfl;
  J.geom[3] = g->glm_alpha;
  return AMRVAC_OK;
}


// Scratch of amrvac_stage_noalloc: the per-kernel path's primitive and
// face-flux buffers, for callers that cannot allocate device memory.  Each
// device holds its own copy from the load of the library's code object until
// the process ends.  Host code reaches it only through the per-device
// address that hipGetSymbolAddress gives (the name itself is a host-side
// stand-in, not a device address); that address is looked up once per
// device, with the device current, by the init entry point.
static __device__ __align__(256) unsigned char scratch[AMRVAC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};
hipError_t g_scratch_err[kScratchDevices] = {};
bool g_scratch_bound[kScratchDevices] = {};

// Look up this device's copy of the scratch array (dev must be current).
void bind_scratch(int dev) {
  if (dev < 0 || dev >= kScratchDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_bound[dev]) return;
  g_scratch_bound[dev] = true;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_scratch_err[dev] = e;
  if (e == hipSuccess)
    g_scratch_ptr[dev] = p;
  else
    (void)hipGetLastError();  // the error is kept here, not left for the next launch check
}

// This device's copy, or null with the lookup's error.
void* scratch_of(int dev, hipError_t* err) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= kScratchDevices || !g_scratch_bound[dev]) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  *err = g_scratch_err[dev];
  return g_scratch_ptr[dev];
}
}  // namespace

thread_local std::string g_init_err;

}  // namespace

struct amrvac_ctx {
  amrvac_grid_desc g{};  // single-job: the grid; batch: shape and physics template
  GridConst G{};
  PhysConst P{};
  FixedBC fixed{};
  bool batch = false;
  int batch_stages = 3;
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<void*> slots;
  int path = AMRVAC_PATH_PLAIN;
  int cap = 0;       // pool places
  int njob_cap = 1;  // job slots
  std::vector<JobRec> jobs;
  std::vector<std::pair<int, int>> free_runs;  // (first, count) of free pool places
  bool dirty = true;
  // device tables (pool-sized) and lists
  int *d_level = nullptr, *d_job = nullptr, *d_link = nullptr, *d_pos = nullptr, *d_wrap = nullptr;
  double* d_invdx = nullptr;
  int *d_order = nullptr, *d_tfill = nullptr, *d_tfused = nullptr, *d_tprol = nullptr, *d_trefl = nullptr;
  size_t cap_order = 0, cap_tfill = 0, cap_tfused = 0, cap_tprol = 0, cap_trefl = 0;
  int n_order = 0, n_tfill = 0, n_tfused = 0, n_tprol = 0, n_trefl = 0;
  int refl_first[3] = {0, 0, 0}, refl_count[3] = {0, 0, 0};  // trefl by direction
  // per-job device arrays
  double* d_geom = nullptr;
  unsigned long long* d_rate = nullptr;
  unsigned int* d_nan = nullptr;
  double* d_jdt = nullptr;  // dt, c_h, kappa of each job slot (library-owned)
  double* d_jch = nullptr;
  double* d_jkappa = nullptr;
  // plain-path scratch (single-job FP64 contexts)
  double* d_prim = nullptr;
  // fused five-cell path in 3D: each cell's x and y flux differences between
  // the stage kernel's two sweeps (single-job FP64 contexts, first use)
  double* d_part = nullptr;
  // fused path of two ghost layers with coarse/fine flux correction: the
  // flux registers the stage fills and the correction reads (first use)
  void* d_freg = nullptr;
  double* d_flux[3] = {nullptr, nullptr, nullptr};
  DevStatus* d_status = nullptr;
  // graph of one step (single-job amrvac_advance)
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_stages = 0;
  int graph_path = -1;
  FusedTune tune{1, 0, 1};  // launch shape of the fused stage
  // CFL rate accumulators (d_rate, d_nan): carry_slot >= 0 means they hold
  // the rate of that slot's current interior, folded in by the fused stage
  // that wrote it; acc_dirty means they may hold anything and must be
  // emptied before the next accumulation.  Otherwise they are empty.
  int carry_slot = -1;
  bool acc_dirty = false;
  // Pinned staging buffers for table uploads (see upload_async).
  static constexpr int kStaging = 8;
  void* stg_host[kStaging] = {};
  size_t stg_cap[kStaging] = {};
  hipEvent_t stg_done[kStaging] = {};
  bool stg_pending[kStaging] = {};
  int stg_next = 0;
  std::string err;

  Tables tables() const { return Tables{d_level, d_job, d_invdx, d_link, d_pos, d_wrap, d_order, n_order}; }
};

namespace {

int fail(amrvac_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIP_TRY(ctx, expr)                                                                 \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail((ctx), AMRVAC_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

void free_all(amrvac_ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  void* ptrs[] = {c->d_level, c->d_job,   c->d_link,  c->d_pos,   c->d_wrap,    c->d_invdx,   c->d_order, c->d_tfill,
                  c->d_tfused, c->d_tprol, c->d_trefl, c->d_geom,  c->d_rate,    c->d_nan,     c->d_jdt,   c->d_jch,
                  c->d_jkappa, c->d_prim,  c->d_flux[0], c->d_flux[1], c->d_flux[2], c->d_status,
                  c->d_part,  c->d_freg};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int k = 0; k < amrvac_ctx::kStaging; ++k) {
    if (c->stg_host[k]) (void)hipHostFree(c->stg_host[k]);
    if (c->stg_done[k]) (void)hipEventDestroy(c->stg_done[k]);
  }
}

int dev_alloc(amrvac_ctx* c, void** p, size_t n) {
  hipError_t e = hipMalloc(p, std::max<size_t>(n, 8));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(c, AMRVAC_E_NOMEM, std::string("hipMalloc of library memory failed: ") + hipGetErrorString(e));
  }
  return AMRVAC_OK;
}

// Host-to-device table uploads ordered on the context's stream: the data is
// copied into a pinned staging buffer and sent with hipMemcpyAsync, so the
// copies queue behind the kernels already enqueued (which still read the old
// tables) and a table change never drains the stream.  A ring of staging
// buffers keeps the host from overwriting one before its copy has run.
struct UploadItem {
  void* dst;
  const void* src;
  size_t bytes;
};

int upload_async(amrvac_ctx* c, const std::vector<UploadItem>& items) {
  auto padded = [](size_t n) { return (n + 255) & ~size_t(255); };
  size_t total = 0;
  for (const auto& it : items) total += padded(it.bytes);
  if (total == 0) return AMRVAC_OK;
  const int k = c->stg_next;
  c->stg_next = (k + 1) % amrvac_ctx::kStaging;
  if (c->stg_pending[k]) {
    HIP_TRY(c, hipEventSynchronize(c->stg_done[k]));
    c->stg_pending[k] = false;
  }
  if (!c->stg_done[k]) HIP_TRY(c, hipEventCreateWithFlags(&c->stg_done[k], hipEventDisableTiming));
  if (c->stg_cap[k] < total) {
    if (c->stg_host[k]) (void)hipHostFree(c->stg_host[k]);
    c->stg_host[k] = nullptr;
    c->stg_cap[k] = 0;
    const size_t n = std::max(total + total / 2, size_t(4096));
    if (hipHostMalloc(&c->stg_host[k], n, hipHostMallocDefault) != hipSuccess) {
      c->stg_host[k] = nullptr;
      return fail(c, AMRVAC_E_NOMEM, "pinned staging allocation failed");
    }
    c->stg_cap[k] = n;
  }
  char* h = static_cast<char*>(c->stg_host[k]);
  size_t off = 0;
  for (const auto& it : items) {
    if (it.bytes == 0) continue;
    std::memcpy(h + off, it.src, it.bytes);
    HIP_TRY(c, hipMemcpyAsync(it.dst, h + off, it.bytes, hipMemcpyHostToDevice, c->stream));
    off += padded(it.bytes);
  }
  HIP_TRY(c, hipEventRecord(c->stg_done[k], c->stream));
  c->stg_pending[k] = true;
  return AMRVAC_OK;
}

// Make room for a host list in a device buffer (growing it by half again
// when needed; a reallocation waits for the stream, since queued kernels may
// still read the old buffer) and add its upload to items.
template <class T>
int stage_list(amrvac_ctx* c, T** d, size_t* capn, const std::vector<T>& h, std::vector<UploadItem>& items) {
  if (h.size() > *capn || !*d) {
    if (*d) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      (void)hipFree(*d);
    }
    *d = nullptr;
    const size_t n = std::max<size_t>(h.size() + h.size() / 2, 64);
    if (int rc = dev_alloc(c, (void**)d, n * sizeof(T))) return rc;
    *capn = n;
  }
  if (!h.empty()) items.push_back(UploadItem{*d, h.data(), h.size() * sizeof(T)});
  return AMRVAC_OK;
}

// Rebuild the active lists and per-job geometry from the job records and
// upload them behind the work already on the stream.  A job is active while
// it has steps left (always, in a single-job context).
int rebuild(amrvac_ctx* c) {
  std::vector<int> order, tfill, tfused, tprol, trefl;
  std::vector<double> geom((size_t)c->njob_cap * 4, 0.0);
  for (int j = 0; j < c->njob_cap; ++j) {
    const JobRec& J = c->jobs[j];
    const bool active = J.used && (!c->batch || J.steps_left > 0);
    if (!active) continue;
    order.insert(order.end(), J.t.order_local.begin(), J.t.order_local.end());
    tfill.insert(tfill.end(), J.t.tfill.begin(), J.t.tfill.end());
    tfused.insert(tfused.end(), J.t.tfused.begin(), J.t.tfused.end());
    tprol.insert(tprol.end(), J.t.tprol.begin(), J.t.tprol.end());
    trefl.insert(trefl.end(), J.t.trefl.begin(), J.t.trefl.end());
    for (int q = 0; q < 4; ++q) geom[4 * j + q] = J.t.geom[q];
  }
  // flux-correction faces grouped by direction (one correction launch each)
  {
    std::vector<int> by_dir;
    by_dir.reserve(trefl.size());
    for (int d = 0; d < 3; ++d) {
      c->refl_first[d] = (int)by_dir.size() / 2;
      for (size_t k = 0; k < trefl.size(); k += 2)
        if ((trefl[k + 1] >> 1) == d) {
          by_dir.push_back(trefl[k]);
          by_dir.push_back(trefl[k + 1]);
        }
      c->refl_count[d] = (int)by_dir.size() / 2 - c->refl_first[d];
    }
    trefl.swap(by_dir);
  }
  int rc;
  std::vector<UploadItem> items;
  if ((rc = stage_list(c, &c->d_order, &c->cap_order, order, items)) ||
      (rc = stage_list(c, &c->d_tfill, &c->cap_tfill, tfill, items)) ||
      (rc = stage_list(c, &c->d_tfused, &c->cap_tfused, tfused, items)) ||
      (rc = stage_list(c, &c->d_tprol, &c->cap_tprol, tprol, items)) ||
      (rc = stage_list(c, &c->d_trefl, &c->cap_trefl, trefl, items)))
    return rc;
  items.push_back(UploadItem{c->d_geom, geom.data(), geom.size() * sizeof(double)});
  if ((rc = upload_async(c, items))) return rc;
  c->n_order = (int)order.size();
  c->n_tfill = (int)tfill.size() / 2;
  c->n_tfused = (int)tfused.size() / 2;
  c->n_tprol = (int)tprol.size() / 2;
  c->n_trefl = (int)trefl.size() / 2;
  c->dirty = false;
  return AMRVAC_OK;
}

void drop_graph(amrvac_ctx* c) {
  if (c->graph_exec) {
    (void)hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
  }
  if (c->graph) {
    (void)hipGraphDestroy(c->graph);
    c->graph = nullptr;
  }
}

// The accumulators no longer describe slot s (it is being written).
void touch_slot(amrvac_ctx* c, int s) {
  if (c->carry_slot == s) {
    c->carry_slot = -1;
    c->acc_dirty = true;
  }
}

// Forget any carried rate (the accumulators must be emptied before use).
void drop_carry(amrvac_ctx* c) {
  if (c->carry_slot >= 0) {
    c->carry_slot = -1;
    c->acc_dirty = true;
  }
}

int ensure_tables(amrvac_ctx* c) {
  if (!c->dirty) return AMRVAC_OK;
  if (c->graph_exec) {  // a replay in flight reads the old lists
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
  }
  drop_carry(c);  // job slots and block lists change
  return rebuild(c);
}

// Copy a job's per-block tables into the pool-sized device tables.
int upload_job_blocks(amrvac_ctx* c, const JobRec& J, int jslot) {
  const size_t f = J.first, n = J.nb;
  std::vector<int> jobv(n, jslot);
  return upload_async(c, {UploadItem{c->d_level + f, J.t.level.data(), n * sizeof(int)},
                          UploadItem{c->d_job + f, jobv.data(), n * sizeof(int)},
                          UploadItem{c->d_pos + 3 * f, J.t.pos.data(), 3 * n * sizeof(int)},
                          UploadItem{c->d_wrap + 3 * f, J.t.wrap.data(), 3 * n * sizeof(int)},
                          UploadItem{c->d_invdx + 3 * f, J.t.invdx.data(), 3 * n * sizeof(double)},
                          UploadItem{c->d_link + f * 6 * LINK_INTS, J.t.link.data(),
                                     n * 6 * LINK_INTS * sizeof(int)}});
}

// Allocate the pool-sized tables and per-job arrays of a new context.
int alloc_context(amrvac_ctx* c) {
  const size_t cap = c->cap, nj = c->njob_cap;
  int rc;
  if ((rc = dev_alloc(c, (void**)&c->d_level, cap * sizeof(int))) ||
      (rc = dev_alloc(c, (void**)&c->d_job, cap * sizeof(int))) ||
      (rc = dev_alloc(c, (void**)&c->d_link, cap * 6 * LINK_INTS * sizeof(int))) ||
      (rc = dev_alloc(c, (void**)&c->d_pos, cap * 3 * sizeof(int))) ||
      (rc = dev_alloc(c, (void**)&c->d_wrap, cap * 3 * sizeof(int))) ||
      (rc = dev_alloc(c, (void**)&c->d_invdx, cap * 3 * sizeof(double))) ||
      (rc = dev_alloc(c, (void**)&c->d_geom, nj * 4 * sizeof(double))) ||
      (rc = dev_alloc(c, (void**)&c->d_rate, nj * sizeof(unsigned long long))) ||
      (rc = dev_alloc(c, (void**)&c->d_nan, nj * sizeof(unsigned int))) ||
      (rc = dev_alloc(c, (void**)&c->d_jdt, nj * sizeof(double))) ||
      (rc = dev_alloc(c, (void**)&c->d_jch, nj * sizeof(double))) ||
      (rc = dev_alloc(c, (void**)&c->d_jkappa, nj * sizeof(double))) ||
      (rc = dev_alloc(c, (void**)&c->d_status, sizeof(DevStatus))))
    return rc;
  HIP_TRY(c, hipMemset(c->d_rate, 0, nj * sizeof(unsigned long long)));
  HIP_TRY(c, hipMemset(c->d_nan, 0, nj * sizeof(unsigned int)));
  HIP_TRY(c, hipMemset(c->d_jdt, 0, nj * sizeof(double)));
  HIP_TRY(c, hipMemset(c->d_jch, 0, nj * sizeof(double)));
  HIP_TRY(c, hipMemset(c->d_jkappa, 0, nj * sizeof(double)));
  HIP_TRY(c, hipMemset(c->d_status, 0, sizeof(DevStatus)));
  HIP_TRY(c, hipMemset(c->d_job, 0, cap * sizeof(int)));
  return AMRVAC_OK;
}

void setup_shape(amrvac_ctx* c, const amrvac_grid_desc* g) {
  c->g = *g;
  GridConst& G = c->G;
  G.ndim = g->ndim;
  G.nx = g->block_nx;
  G.ng = g->nghost;
  G.pn = G.nx + 2 * G.ng;
  G.nb = c->cap;
  G.nfaces = (G.nx + 1) * G.nx * (G.ndim == 3 ? G.nx : 1);
  G.pcells = (long)G.pn * G.pn * (G.ndim == 3 ? G.pn : 1);
  G.icells = (long)G.nx * G.nx * (G.ndim == 3 ? G.nx : 1);
  G.precision = g->precision;
  c->P = PhysConst{g->gamma, g->gamma - 1.0, 1.0 / (g->gamma - 1.0), g->small_density, g->small_pressure,
                   g->fix_small_values, g->limiter, g->flux};
  std::memcpy(c->fixed.prim, g->bc_fixed_prim, sizeof(c->fixed.prim));
  if (g->precision == AMRVAC_FP32_MIXED) c->path = AMRVAC_PATH_FUSED;
}

int check_slot(amrvac_ctx* c, int s) {
  if (s < 0 || s >= (int)c->slots.size()) return fail(c, AMRVAC_E_ARG, "slot index out of range");
  return AMRVAC_OK;
}

int fill_slot(amrvac_ctx* c, int slot) {
  const Tables T = c->tables();
  const bool fused = c->path == AMRVAC_PATH_FUSED;
  HIP_TRY(c, launch_fill_faces(c->stream, c->G, fused ? c->d_tfused : c->d_tfill, fused ? c->n_tfused : c->n_tfill,
                               T, c->slots[slot], c->P, c->fixed));
  HIP_TRY(c, launch_prolong_faces(c->stream, c->G, c->d_tprol, c->n_tprol, T, c->slots[slot]));
  return AMRVAC_OK;
}

JobCfl cfl_state(amrvac_ctx* c, double* dt, double* ch, double* kappa) {
  return JobCfl{c->d_rate, c->d_nan, c->d_geom, dt, ch, kappa, c->njob_cap};
}

// The fused stage can fold the next step's CFL rate into its output only
// where nothing changes that output afterwards: with coarse/fine flux
// correction the stage leaves out the cells next to faces towards finer
// leaves, and a pass after the correction folds those in.  The 3D stage
// with three ghost layers does not fold: on 256^3 a step with the folding
// instance and no separate CFL pass was no faster in FP64 and 0.3 ms slower
// in FP32-mixed (the update's extra live state at 168 VGPRs).
bool can_carry(const amrvac_ctx* c) {
  return c->path == AMRVAC_PATH_FUSED && !(c->G.ng == 3 && c->G.ndim == 3);
}

// flux registers for the fused stage, when a coarse/fine correction follows
// it (else null)
void* stage_freg(const amrvac_ctx* c) {
  return c->path == AMRVAC_PATH_FUSED && c->n_trefl > 0 ? c->d_freg : nullptr;
}

int clear_if_dirty(amrvac_ctx* c) {
  if (c->acc_dirty) {
    HIP_TRY(c, launch_cfl_clear(c->stream, cfl_state(c, nullptr, nullptr, nullptr)));
    c->acc_dirty = false;
  }
  return AMRVAC_OK;
}

// dt, c_h, kappa from slot: only the finalize kernel when the accumulators
// carry slot's rate, else empty them if needed, accumulate and finalize.
int cfl_of_slot(amrvac_ctx* c, int slot, double* dt, double* ch, double* kap) {
  const JobCfl C = cfl_state(c, dt, ch, kap);
  if (c->carry_slot != slot) {
    drop_carry(c);
    if (int rc = clear_if_dirty(c)) return rc;
    HIP_TRY(c, launch_cfl_accumulate(c->stream, c->G, c->tables(), c->slots[slot], c->P, c->d_status, C));
  }
  HIP_TRY(c, launch_cfl_finalize(c->stream, c->d_status, C));
  c->carry_slot = -1;
  c->acc_dirty = false;
  return AMRVAC_OK;
}

// The per-kernel (plain) FP64 stage on the given primitive and face-flux
// scratch: conserved -> primitive over interior and face ghost cells, face
// fluxes per direction, flux correction at coarse/fine faces, update.
int plain_stage(amrvac_ctx* c, int in, int base, int out, double w, const JobScalars& J, double* prim,
                double* const flux[3]) {
  const Tables T = c->tables();
  HIP_TRY(c, launch_prim(c->stream, c->G, c->slots[in], prim, c->P, c->d_status));
  for (int d = 0; d < c->G.ndim; ++d)
    HIP_TRY(c, launch_flux(c->stream, c->G, d, prim, flux[d], J.ch, c->P, T.inv_dx));
  FluxPtrs fp{{flux[0], flux[1], flux[2]}};
  HIP_TRY(c, launch_reflux(c->stream, c->G, c->d_trefl, c->n_trefl, T, fp));
  HIP_TRY(c, launch_update(c->stream, c->G, T, c->slots[in], c->slots[base], c->slots[out], w, fp, J.dt, J.dt_scale,
                           J.kappa));
  return AMRVAC_OK;
}

// fold_cfl: on the fused path without flux corrections, also leave the CFL
// rate of out in the accumulators (carry_slot = out).
int stage_any(amrvac_ctx* c, int in, int base, int out, double w, const JobScalars& J, bool fold_cfl = false) {
  const Tables T = c->tables();
  touch_slot(c, out);
  if (c->path == AMRVAC_PATH_FUSED) {
    const bool fold = fold_cfl && can_carry(c);
    const bool corr = c->n_trefl > 0;
    void* freg = stage_freg(c);
    JobCfl C{};
    if (fold) {
      drop_carry(c);
      if (int rc = clear_if_dirty(c)) return rc;
      C = cfl_state(c, nullptr, nullptr, nullptr);
      C.skip_fine = corr ? 1 : 0;
    }
    if (c->G.ng == 3)
      HIP_TRY(c, launch_fused5_stage(c->stream, c->G, T, J, c->slots[in], c->slots[base], c->slots[out], w, c->P,
                                     c->d_status, c->d_part, freg, fold ? &C : nullptr));
    else
      HIP_TRY(c, launch_fused_stage(c->stream, c->G, T, J, c->tune, c->slots[in], c->slots[base], c->slots[out], w,
                                    c->P, c->d_status, fold ? &C : nullptr, freg));
    HIP_TRY(c, launch_reflux_apply(c->stream, c->G, T, J, c->d_trefl, c->refl_first, c->refl_count,
                                   c->slots[out], w, freg));
    if (fold && corr)
      HIP_TRY(c, launch_cfl_reflux_cells(c->stream, c->G, T, c->d_trefl, c->n_trefl, c->slots[out], c->P,
                                         c->d_status, C));
    if (fold) c->carry_slot = out;
    return AMRVAC_OK;
  }
  return plain_stage(c, in, base, out, w, J, c->d_prim, c->d_flux);
}

// cfl -> [fill -> stage] x nstages on slots 0, 1, 2 with per-job scalars;
// the last stage folds the next step's CFL rate in where it can, so the next
// step's cfl is only the finalize kernel.
int enqueue_step(amrvac_ctx* c, int nstages, double* dt, double* ch, double* kap) {
  if (int rc = cfl_of_slot(c, 0, dt, ch, kap)) return rc;
  const JobScalars J{dt, ch, kap};
  int rc;
  if (nstages == 2) {
    if ((rc = fill_slot(c, 0)) || (rc = stage_any(c, 0, 0, 1, 1.0, J))) return rc;
    if ((rc = fill_slot(c, 1)) || (rc = stage_any(c, 1, 0, 0, 0.5, J, true))) return rc;
    return AMRVAC_OK;
  }
  if (nstages == 3) {
    if ((rc = fill_slot(c, 0)) || (rc = stage_any(c, 0, 0, 1, 1.0, J))) return rc;
    if ((rc = fill_slot(c, 1)) || (rc = stage_any(c, 1, 0, 2, 0.25, J))) return rc;
    if ((rc = fill_slot(c, 2)) || (rc = stage_any(c, 2, 0, 0, 2.0 / 3.0, J, true))) return rc;
    return AMRVAC_OK;
  }
  if (nstages == 4) {
    // SSPRK(4,3): four stages of dt/2; u3 = u0 + (1/3)((u2 + h L(u2)) - u0)
    JobScalars H = J;
    H.dt_scale = 0.5;
    if ((rc = fill_slot(c, 0)) || (rc = stage_any(c, 0, 0, 1, 1.0, H))) return rc;
    if ((rc = fill_slot(c, 1)) || (rc = stage_any(c, 1, 1, 2, 1.0, H))) return rc;
    if ((rc = fill_slot(c, 2)) || (rc = stage_any(c, 2, 0, 1, 1.0 / 3.0, H))) return rc;
    if ((rc = fill_slot(c, 1)) || (rc = stage_any(c, 1, 1, 0, 1.0, H, true))) return rc;
    return AMRVAC_OK;
  }
  // SSPRK(5,4) of Spiteri and Ruuth, Shu-Osher coefficients (alpha_kj for
  // states, beta_kj for dt L; each row's alphas sum to one):
  //   u1 = u0 + b10 dt L(u0)
  //   u_k = u0 + a_k,k-1 ((u_k-1 + (b_k,k-1/a_k,k-1) dt L(u_k-1)) - u0),  k = 2, 3, 4
  //   u5 = a52 u2 + a53 u3 + b53 dt L(u3) + a54 u4 + b54 dt L(u4)
  // The fourth row gives dt L(u3) = ((u4 - u0) - a43 (u3 - u0)) / b43, so
  //   u5 = u0 + g2 (u2 - u0) + g3 (u3 - u0) + g4 (u4 - u0) + b54 dt L(u4)
  // with g2 = a52, g3 = a53 - b53 a43 / b43, g4 = a54 + b53 / b43.  g3 is zero
  // for this scheme (the published 15-digit values give -1.8e-16), so the
  // fifth stage is a stage from u4 with weight g4 and scale b54 / g4 whose
  // base is u0 + (g2 / (1 - g4)) (u2 - u0).  Slots: u0 0, u1 1, u2 2, u3 1,
  // u4 3, fifth-stage base 1.
  constexpr double b10 = 0.391752226571890;
  constexpr double a21 = 0.555629506348765, b21 = 0.368410593050371;
  constexpr double a32 = 0.379898148511597, b32 = 0.251891774271694;
  constexpr double a43 = 0.821920045606868, b43 = 0.544974750228521;
  constexpr double a52 = 0.517231671970585, b53 = 0.063692468666290;
  constexpr double a54 = 0.386708617503269, b54 = 0.226007483236906;
  constexpr double g4 = a54 + b53 / b43;
  constexpr double c2 = a52 / (1.0 - g4);
  JobScalars S = J;
  S.dt_scale = b10;
  if ((rc = fill_slot(c, 0)) || (rc = stage_any(c, 0, 0, 1, 1.0, S))) return rc;
  S.dt_scale = b21 / a21;
  if ((rc = fill_slot(c, 1)) || (rc = stage_any(c, 1, 0, 2, a21, S))) return rc;
  S.dt_scale = b32 / a32;
  if ((rc = fill_slot(c, 2)) || (rc = stage_any(c, 2, 0, 1, a32, S))) return rc;
  S.dt_scale = b43 / a43;
  if ((rc = fill_slot(c, 1)) || (rc = stage_any(c, 1, 0, 3, a43, S))) return rc;
  touch_slot(c, 1);
  HIP_TRY(c, launch_combine(c->stream, c->G, c->tables(), c->slots[0], c->slots[2], c2, c->slots[1]));
  S.dt_scale = b54 / g4;
  if ((rc = fill_slot(c, 3)) || (rc = stage_any(c, 3, 1, 0, g4, S, true))) return rc;
  return AMRVAC_OK;
}

int slots_for_stages(int nstages) { return nstages >= 5 ? 4 : (nstages >= 3 ? 3 : 2); }

// The plain (per-kernel) FP64 path's primitive and face-flux scratch, the
// 3D five-cell fused stage's array of in-plane flux differences, and the
// flux registers of the fused path on grids with coarse/fine flux
// correction (110 KB per 16^3 block in FP64), allocated on
// first use of their path: a context that only runs the fused path on a
// uniform grid holds none of them (the plain scratch for 4096 blocks of
// 16^3 is 6 GB, the difference array 1.2 GB).  Called by the entry points
// before they enqueue work, so never inside a graph capture.
int ensure_plain_scratch(amrvac_ctx* c) {
  if (c->path == AMRVAC_PATH_FUSED && c->n_trefl > 0 && !c->d_freg) {
    const size_t nfc = c->G.ndim == 3 ? (size_t)c->G.nx * c->G.nx : (size_t)c->G.nx;
    const size_t rbytes = c->G.precision == 0 ? sizeof(double) : sizeof(float);
    if (int rc = dev_alloc(c, &c->d_freg, (size_t)c->cap * 6 * NV * nfc * rbytes)) return rc;
  }
  if (c->path == AMRVAC_PATH_FUSED && c->G.ng == 3 && c->G.ndim == 3 && !c->d_part)
    if (int rc = dev_alloc(c, (void**)&c->d_part, (size_t)c->cap * NV * c->G.icells * sizeof(double))) return rc;
  if (c->path != AMRVAC_PATH_PLAIN || c->d_prim) return AMRVAC_OK;
  const size_t nb = (size_t)c->cap;
  const size_t pcs = nb * NV * c->G.pcells * sizeof(double);
  const size_t fcs = nb * NV * c->G.nfaces * sizeof(double);
  if (int rc = dev_alloc(c, (void**)&c->d_prim, pcs)) return rc;
  for (int d = 0; d < c->G.ndim; ++d)
    if (int rc = dev_alloc(c, (void**)&c->d_flux[d], fcs)) return rc;
  return AMRVAC_OK;
}

// Argument checks shared by the stage entry points (base becomes out when
// w == 1, where it is not read).
int stage_args(amrvac_ctx* c, int in, int* base, int out, double w, const double* dt_dev, const double* ch_dev,
               const double* kappa_dev) {
  if (c->batch) return fail(c, AMRVAC_E_STATE, "batch contexts step with amrvac_batch_step");
  if (int rc = check_slot(c, in)) return rc;
  if (int rc = check_slot(c, out)) return rc;
  if (w != 1.0) {
    if (int rc = check_slot(c, *base)) return rc;
  } else {
    *base = out;
  }
  if (in == out) return fail(c, AMRVAC_E_ARG, "in and out slots must differ");
  if (*base == in && w != 1.0) return fail(c, AMRVAC_E_ARG, "base must differ from in");
  if (!dt_dev || !ch_dev || !kappa_dev) return fail(c, AMRVAC_E_ARG, "null dt/c_h/kappa pointer");
  if (!(w > 0.0 && w <= 1.0)) return fail(c, AMRVAC_E_ARG, "stage weight must be in (0, 1]");
  return AMRVAC_OK;
}

int stage_entry(amrvac_ctx* c, int in, int base, int out, double w, const double* dt_dev, const double* ch_dev,
                const double* kappa_dev, bool fold_cfl) {
  if (!c) return AMRVAC_E_ARG;
  if (int rc = stage_args(c, in, &base, out, w, dt_dev, ch_dev, kappa_dev)) return rc;
  if (int rc = ensure_tables(c)) return rc;
  if (int rc = ensure_plain_scratch(c)) return rc;
  return stage_any(c, in, base, out, w, JobScalars{dt_dev, ch_dev, kappa_dev}, fold_cfl);
}

bool job_ok(const amrvac_ctx* c, int job) { return c->batch && job >= 0 && job < c->njob_cap && c->jobs[job].used; }

}  // namespace

namespace {

// A single-job context on caller-owned slots (amrvac_init_blocks, and the
// new context of a regrid).
int create_single(amrvac_ctx** out, const amrvac_grid_desc* g, int nb, const int* level, const int* ijk,
                  void* const* slots, int nslots, void* stream) {
  if (!out) return AMRVAC_E_ARG;
  *out = nullptr;
  std::string why;
  if (check_desc(g, &why) != AMRVAC_OK) { g_init_err = why; return AMRVAC_E_ARG; }
  if (nb < 1 || !level || !ijk || !slots || nslots < 1) { g_init_err = "need blocks, tables and slots"; return AMRVAC_E_ARG; }
  for (int s = 0; s < nslots; ++s)
    if (!slots[s]) { g_init_err = "null slot pointer"; return AMRVAC_E_ARG; }
  JobRec J;
  if (build_job(g, nb, level, ijk, 0, &J.t) != AMRVAC_OK) { g_init_err = J.t.err; return AMRVAC_E_ARG; }

  amrvac_ctx* c = new amrvac_ctx();
  c->cap = nb;
  c->njob_cap = 1;
  setup_shape(c, g);
  c->stream = static_cast<hipStream_t>(stream);
  c->slots.clear();
  for (int k = 0; k < nslots; ++k) c->slots.push_back(static_cast<char*>(slots[k]) + slot_lead(g->precision));
  (void)hipGetDevice(&c->device);
  bind_scratch(c->device);
  J.used = true;
  J.first = 0;
  J.nb = nb;
  c->jobs.push_back(std::move(J));
  int rc = alloc_context(c);
  if (!rc) rc = upload_job_blocks(c, c->jobs[0], 0);
  if (!rc) rc = rebuild(c);
  if (!rc) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) rc = fail(c, AMRVAC_E_HIP, std::string("init: ") + hipGetErrorString(e));
  }
  if (rc) {
    g_init_err = c->err;
    free_all(c);
    delete c;
    return rc;
  }
  *out = c;
  return AMRVAC_OK;
}

// Leaf-set planning for a regrid (host only).  Slots of a level are block
// positions; a slot is covered by the leaf at or above it.
struct Planner {
  int ndim = 2;
  long base[3] = {1, 1, 1};
  bool per[3] = {false, false, false};
  KeySet leaves;

  long nblk(int l, int d) const { return d < ndim ? base[d] << (l - 1) : 1; }
  // wrap q into the domain of level l; false outside a non-periodic side
  bool wrap(int l, long q[3]) const {
    for (int d = 0; d < ndim; ++d)
      if (q[d] < 0 || q[d] >= nblk(l, d)) {
        if (!per[d]) return false;
        q[d] = (q[d] + nblk(l, d)) % nblk(l, d);
      }
    return true;
  }
  // level of the leaf covering slot q of level l, 0 if the slot is refined
  int cover(int l, const long q[3]) const {
    long p[3] = {q[0], q[1], q[2]};
    for (int m = l; m >= 1; --m) {
      if (leaves.count(KeyL{m, p[0], p[1], p[2]})) return m;
      for (int d = 0; d < 3; ++d) p[d] >>= 1;
    }
    return 0;
  }
  KeyL cover_key(int l, const long q[3]) const {
    long p[3] = {q[0], q[1], q[2]};
    for (int m = l; m >= 1; --m) {
      const KeyL k{m, p[0], p[1], p[2]};
      if (leaves.count(k)) return k;
      for (int d = 0; d < 3; ++d) p[d] >>= 1;
    }
    return KeyL{0, 0, 0, 0};
  }
  // replace leaf k by its children; the children are appended to *born
  void refine(const KeyL& k, std::vector<KeyL>* born) {
    leaves.erase(k);
    for (int cz = 0; cz < (ndim == 3 ? 2 : 1); ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          const KeyL c{k.l + 1, 2 * k.i + cx, 2 * k.j + cy, ndim == 3 ? 2 * k.k + cz : 0};
          leaves.insert(c);
          born->push_back(c);
        }
  }
  template <class F>
  void for_neighbours(const KeyL& k, F f) const {
    for (int oz = (ndim == 3 ? -1 : 0); oz <= (ndim == 3 ? 1 : 0); ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          if (!ox && !oy && !oz) continue;
          long q[3] = {k.i + ox, k.j + oy, k.k + oz};
          if (!wrap(k.l, q)) continue;
          const long off[3] = {ox, oy, oz};
          f(q, off);
        }
  }
  // refine leaves that are two levels coarser than a neighbour of a leaf.
  // The input set was 2:1 nested, so a violation needs a new leaf on its
  // fine side: only the leaves born by refinement (and those born while
  // restoring) are examined, as a work list.
  void nest(std::vector<KeyL> work) {
    while (!work.empty()) {
      const KeyL k = work.back();
      work.pop_back();
      if (!leaves.count(k)) continue;  // refined again meanwhile
      for_neighbours(k, [&](const long q[3], const long*) {
        const int m = cover(k.l, q);
        if (m != 0 && m < k.l - 1) {
          const KeyL t = cover_key(k.l, q);
          if (leaves.count(t)) refine(t, &work);
        }
      });
      // (a refinement above may have coarse neighbours of its own: its
      // children are on the work list)
    }
  }
  // would the leaf parent (replacing its children) be next to a leaf two
  // levels finer?
  bool coarsening_ok(const KeyL& par) const {
    bool ok = true;
    for_neighbours(par, [&](const long q[3], const long* off) {
      if (!ok || cover(par.l, q) != 0) return;
      // slot q is refined: its children next to par must be leaves
      for (int cz = 0; cz < (ndim == 3 ? 2 : 1); ++cz)
        for (int cy = 0; cy < 2; ++cy)
          for (int cx = 0; cx < 2; ++cx) {
            const long cc[3] = {cx, cy, cz};
            bool adjacent = true;
            for (int d = 0; d < ndim; ++d) {
              if (off[d] == 1 && cc[d] != 0) adjacent = false;
              if (off[d] == -1 && cc[d] != 1) adjacent = false;
            }
            if (!adjacent) continue;
            const long c[3] = {2 * q[0] + cx, 2 * q[1] + cy, ndim == 3 ? 2 * q[2] + cz : 0};
            if (!leaves.count(KeyL{par.l + 1, c[0], c[1], c[2]})) ok = false;
          }
    });
    return ok;
  }
};

}  // namespace

extern "C" {

int amrvac_slot_bytes(const amrvac_grid_desc* g, int nblocks, size_t* bytes) {
  std::string why;
  if (check_desc(g, &why) != AMRVAC_OK || nblocks < 1 || !bytes) return AMRVAC_E_ARG;
  *bytes = (size_t)slot_bytes_of(g, nblocks);
  return AMRVAC_OK;
}

const char* amrvac_last_error(const amrvac_ctx* c) {
  if (!c) return g_init_err.c_str();
  return c->err.c_str();
}

int amrvac_destroy(amrvac_ctx* c) {
  if (!c) return AMRVAC_E_ARG;
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
  return AMRVAC_OK;
}

int amrvac_init_blocks(amrvac_ctx** out, const amrvac_grid_desc* g, int nb, const int* level, const int* ijk,
                       void* const* slots, int nslots, void* stream) {
  return create_single(out, g, nb, level, ijk, slots, nslots, stream);
}

int amrvac_set_primitive(amrvac_ctx* c, int slot, const double* prim_dev) {
  if (!c) return AMRVAC_E_ARG;
  if (c->batch) return fail(c, AMRVAC_E_STATE, "batch contexts take initial states in amrvac_batch_add_job");
  if (int rc = check_slot(c, slot)) return rc;
  if (!prim_dev) return fail(c, AMRVAC_E_ARG, "null primitive array");
  touch_slot(c, slot);
  HIP_TRY(c, launch_set_prim(c->stream, c->G, 0, c->cap, prim_dev, c->slots[slot], c->P));
  return AMRVAC_OK;
}

int amrvac_get_conserved(amrvac_ctx* c, int slot, double* cons_dev) {
  if (!c) return AMRVAC_E_ARG;
  if (c->batch) return fail(c, AMRVAC_E_STATE, "use amrvac_batch_get_job on batch contexts");
  if (int rc = check_slot(c, slot)) return rc;
  if (!cons_dev) return fail(c, AMRVAC_E_ARG, "null output array");
  HIP_TRY(c, launch_get_cons(c->stream, c->G, 0, c->cap, c->slots[slot], cons_dev));
  return AMRVAC_OK;
}

int amrvac_fill_ghosts(amrvac_ctx* c, int slot) {
  if (!c) return AMRVAC_E_ARG;
  if (int rc = check_slot(c, slot)) return rc;
  if (int rc = ensure_tables(c)) return rc;
  return fill_slot(c, slot);
}

int amrvac_cfl_dt(amrvac_ctx* c, int slot, double* dt_dev, double* ch_dev, double* kappa_dev) {
  if (!c) return AMRVAC_E_ARG;
  if (c->batch) return fail(c, AMRVAC_E_STATE, "batch contexts compute per-job dt in amrvac_batch_step");
  if (int rc = check_slot(c, slot)) return rc;
  if (!dt_dev || !ch_dev || !kappa_dev) return fail(c, AMRVAC_E_ARG, "null dt/c_h/kappa pointer");
  if (int rc = ensure_tables(c)) return rc;
  return cfl_of_slot(c, slot, dt_dev, ch_dev, kappa_dev);
}


int amrvac_stage(amrvac_ctx* c, int in, int base, int out, double w, const double* dt_dev, const double* ch_dev,
                 const double* kappa_dev) {
  return stage_entry(c, in, base, out, w, dt_dev, ch_dev, kappa_dev, false);
}

int amrvac_stage_cfl(amrvac_ctx* c, int in, int base, int out, double w, const double* dt_dev, const double* ch_dev,
                     const double* kappa_dev) {
  return stage_entry(c, in, base, out, w, dt_dev, ch_dev, kappa_dev, true);
}

int amrvac_stage_noalloc(amrvac_ctx* c, int in, int base, int out, double w, const double* dt_dev,
                         const double* ch_dev, const double* kappa_dev) {
  if (!c) return AMRVAC_E_ARG;
  if (c->g.precision != AMRVAC_FP64)
    return fail(c, AMRVAC_E_ARG, "amrvac_stage_noalloc runs the per-kernel FP64 path: FP64 contexts only");
  if (int rc = stage_args(c, in, &base, out, w, dt_dev, ch_dev, kappa_dev)) return rc;
  if (c->dirty) return fail(c, AMRVAC_E_STATE, "the block tables need a rebuild, which allocates");
  // primitives of every padded cell, then the face fluxes of each direction,
  // each part starting on a 256-byte boundary
  const size_t prim_bytes = ((size_t)c->G.nb * NV * c->G.pcells * sizeof(double) + 255) & ~(size_t)255;
  const size_t flux_bytes = ((size_t)c->G.nb * NV * c->G.nfaces * sizeof(double) + 255) & ~(size_t)255;
  const size_t need = prim_bytes + (size_t)c->G.ndim * flux_bytes;
  if (need > (size_t)AMRVAC_NOALLOC_SCRATCH_BYTES)
    return fail(c, AMRVAC_E_ARG,
                "amrvac_stage_noalloc: this grid needs " + std::to_string(need) +
                    " bytes of scratch, more than the static array's " +
                    std::to_string((size_t)AMRVAC_NOALLOC_SCRATCH_BYTES) + " (AMRVAC_NOALLOC_SCRATCH_BYTES)");
  hipError_t e;
  char* p = static_cast<char*>(scratch_of(c->device, &e));
  if (!p) return fail(c, AMRVAC_E_HIP, std::string("static scratch address not available: ") + hipGetErrorString(e));
  double* flux[3] = {nullptr, nullptr, nullptr};
  for (int d = 0; d < c->G.ndim; ++d) flux[d] = reinterpret_cast<double*>(p + prim_bytes + (size_t)d * flux_bytes);
  touch_slot(c, out);
  return plain_stage(c, in, base, out, w, JobScalars{dt_dev, ch_dev, kappa_dev}, reinterpret_cast<double*>(p), flux);
}

int amrvac_combine(amrvac_ctx* c, int a, int b, double coef, int out) {
  if (!c) return AMRVAC_E_ARG;
  if (c->batch) return fail(c, AMRVAC_E_STATE, "batch contexts step with amrvac_batch_step");
  if (int rc = check_slot(c, a)) return rc;
  if (int rc = check_slot(c, b)) return rc;
  if (int rc = check_slot(c, out)) return rc;
  if (!std::isfinite(coef)) return fail(c, AMRVAC_E_ARG, "non-finite combination coefficient");
  if (int rc = ensure_tables(c)) return rc;
  touch_slot(c, out);
  HIP_TRY(c, launch_combine(c->stream, c->G, c->tables(), c->slots[a], c->slots[b], coef, c->slots[out]));
  return AMRVAC_OK;
}

int amrvac_lohner(amrvac_ctx* c, int slot, const double* weights, double wavefilter, double* indicator_dev) {
  if (!c) return AMRVAC_E_ARG;
  if (c->batch) return fail(c, AMRVAC_E_STATE, "batch contexts have no per-context block indicator");
  if (int rc = check_slot(c, slot)) return rc;
  if (!weights || !indicator_dev) return fail(c, AMRVAC_E_ARG, "null weights or indicator pointer");
  LohnerParams L{};
  bool any = false;
  for (int q = 0; q < NV; ++q) {
    if (!(weights[q] >= 0.0) || !std::isfinite(weights[q])) return fail(c, AMRVAC_E_ARG, "weights must be finite and >= 0");
    L.weight[q] = weights[q];
    any = any || weights[q] > 0.0;
  }
  if (!any) return fail(c, AMRVAC_E_ARG, "at least one weight must be positive");
  if (!(wavefilter >= 0.0) || !std::isfinite(wavefilter)) return fail(c, AMRVAC_E_ARG, "wavefilter must be finite and >= 0");
  L.wavefilter = wavefilter;
  if (int rc = ensure_tables(c)) return rc;
  if (int rc = fill_slot(c, slot)) return rc;
  HIP_TRY(c, launch_lohner(c->stream, c->G, c->tables(), c->slots[slot], L, indicator_dev));
  return AMRVAC_OK;
}

int amrvac_regrid_plan(const amrvac_grid_desc* g, int nb, const int* level, const int* ijk, const int* flags,
                       int max_level, int cap, int* nb_new, int* level_out, int* ijk_out) {
  if (!g || !level || !ijk || !flags || !nb_new || nb < 1) return AMRVAC_E_ARG;
  std::string why;
  if (check_desc(g, &why) != AMRVAC_OK) { g_init_err = why; return AMRVAC_E_ARG; }
  JobBuild J;
  if (build_job(g, nb, level, ijk, 0, &J) != AMRVAC_OK) { g_init_err = J.err; return AMRVAC_E_ARG; }
  Planner P;
  P.ndim = g->ndim;
  for (int d = 0; d < 3; ++d) {
    P.base[d] = d < P.ndim ? g->base_blocks[d] : 1;
    P.per[d] = d < P.ndim && g->bc_lo[d] == AMRVAC_BC_PERIODIC;
  }
  const int lmax = std::min(std::max(max_level, 1), MAXLEV);
  KeyMap old;
  old.reserve((size_t)nb * 2);
  P.leaves.reserve((size_t)nb * 4);
  for (int b = 0; b < nb; ++b) {
    const KeyL k{J.level[b], J.pos[3 * b], J.pos[3 * b + 1], J.pos[3 * b + 2]};
    old[k] = b;
    P.leaves.insert(k);
  }
  std::vector<KeyL> born;
  for (const auto& kv : old)
    if (flags[kv.second] > 0 && kv.first.l < lmax) P.refine(kv.first, &born);
  P.nest(std::move(born));
  // coarsen complete sibling sets of old leaves that are all flagged, one
  // parent at a time, where nesting allows
  KeySet parents;
  for (const auto& kv : old)
    if (flags[kv.second] < 0 && kv.first.l > 1)
      parents.insert(KeyL{kv.first.l - 1, kv.first.i >> 1, kv.first.j >> 1, kv.first.k >> 1});
  // (repeated until nothing changes: a set blocked by a finer neighbour set
  // merges once that set has merged)
  for (bool changed = true; changed;) {
    changed = false;
    for (auto pit = parents.begin(); pit != parents.end();) {
      const KeyL par = *pit;
      std::vector<KeyL> kids;
      bool all = true;
      for (int cz = 0; cz < (P.ndim == 3 ? 2 : 1) && all; ++cz)
        for (int cy = 0; cy < 2 && all; ++cy)
          for (int cx = 0; cx < 2 && all; ++cx) {
            const KeyL k{par.l + 1, 2 * par.i + cx, 2 * par.j + cy, P.ndim == 3 ? 2 * par.k + cz : 0};
            auto it = old.find(k);
            if (it == old.end() || flags[it->second] >= 0 || !P.leaves.count(k)) all = false;
            kids.push_back(k);
          }
      if (!all) {
        pit = parents.erase(pit);  // never mergeable
        continue;
      }
      if (!P.coarsening_ok(par)) {
        ++pit;
        continue;
      }
      for (const KeyL& k : kids) P.leaves.erase(k);
      P.leaves.insert(par);
      pit = parents.erase(pit);
      changed = true;
    }
  }
  *nb_new = (int)P.leaves.size();
  if (!level_out || !ijk_out || cap < *nb_new) return AMRVAC_E_NOMEM;
  // (sorted by level, then position: the output does not depend on the
  // hash containers' iteration order)
  std::vector<KeyL> sorted(P.leaves.begin(), P.leaves.end());
  std::sort(sorted.begin(), sorted.end());
  int n = 0;
  for (const KeyL& k : sorted) {
    level_out[n] = k.l;
    ijk_out[3 * n] = (int)k.i;
    ijk_out[3 * n + 1] = (int)k.j;
    ijk_out[3 * n + 2] = (int)k.k;
    ++n;
  }
  return AMRVAC_OK;
}

int amrvac_regrid(amrvac_ctx* c, int slot, int nb, const int* level, const int* ijk, void* const* slots, int nslots,
                  amrvac_ctx** out) {
  if (!out) return AMRVAC_E_ARG;
  *out = nullptr;
  if (!c) return AMRVAC_E_ARG;
  if (c->batch) return fail(c, AMRVAC_E_STATE, "regrid needs a single-job context");
  if (int rc = check_slot(c, slot)) return rc;
  if (nb < 1 || !level || !ijk) return fail(c, AMRVAC_E_ARG, "regrid needs a block table");
  // transfer tasks from the old leaf set
  const JobBuild& J = c->jobs[0].t;
  const int ndim = c->g.ndim;
  KeyMap old;
  old.reserve(J.level.size() * 2);
  for (int b = 0; b < (int)J.level.size(); ++b) old[KeyL{J.level[b], J.pos[3 * b], J.pos[3 * b + 1], J.pos[3 * b + 2]}] = b;
  std::vector<int> tasks((size_t)nb * REGRID_TASK_INTS, 0);
  for (int n = 0; n < nb; ++n) {
    int* T = &tasks[(size_t)n * REGRID_TASK_INTS];
    const long p[3] = {ijk[3 * n], ijk[3 * n + 1], ndim == 3 ? ijk[3 * n + 2] : 0};
    const int l = level[n];
    T[1] = n;
    auto it = old.find(KeyL{l, p[0], p[1], p[2]});
    if (it != old.end()) {
      T[0] = REGRID_COPY;
      T[2] = it->second;
      continue;
    }
    auto ip = l > 1 ? old.find(KeyL{l - 1, p[0] >> 1, p[1] >> 1, p[2] >> 1}) : old.end();
    if (ip != old.end()) {
      T[0] = REGRID_PROLONG;
      T[2] = ip->second;
      for (int d = 0; d < 3; ++d) T[3 + d] = (int)(p[d] & 1);
      continue;
    }
    T[0] = REGRID_RESTRICT;
    for (int cz = 0; cz < (ndim == 3 ? 2 : 1); ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          auto ic = old.find(KeyL{l + 1, 2 * p[0] + cx, 2 * p[1] + cy, ndim == 3 ? 2 * p[2] + cz : 0});
          if (ic == old.end())
            return fail(c, AMRVAC_E_ARG, "regrid block is not an old block, a child of an old leaf or a parent of old leaves");
          T[2 + cx + 2 * cy + 4 * cz] = ic->second;
        }
  }
  amrvac_ctx* nc = nullptr;
  if (int rc = create_single(&nc, &c->g, nb, level, ijk, slots, nslots, c->stream))
    return fail(c, rc, "regrid: " + g_init_err);
  nc->tune = c->tune;
  int rc = AMRVAC_OK;
  if (nc->path != c->path) rc = amrvac_set_path(nc, c->path);
  if (!rc) rc = ensure_tables(c);
  if (!rc) rc = fill_slot(c, slot);
  int* d_tasks = nullptr;
  const size_t bytes = tasks.size() * sizeof(int);
  if (!rc && hipMalloc(&d_tasks, bytes) != hipSuccess) rc = fail(c, AMRVAC_E_NOMEM, "regrid task buffer");
  if (!rc && hipMemcpyAsync(d_tasks, tasks.data(), bytes, hipMemcpyHostToDevice, c->stream) != hipSuccess)
    rc = fail(c, AMRVAC_E_HIP, "regrid task upload");
  if (!rc && launch_regrid(c->stream, c->G, c->tables(), d_tasks, nb, c->slots[slot], nc->slots[0]) != hipSuccess)
    rc = fail(c, AMRVAC_E_HIP, "regrid transfer launch");
  const hipError_t e = hipStreamSynchronize(c->stream);
  if (!rc && e != hipSuccess) rc = fail(c, AMRVAC_E_HIP, std::string("regrid: ") + hipGetErrorString(e));
  if (d_tasks) (void)hipFree(d_tasks);
  if (rc) {
    amrvac_destroy(nc);
    return rc;
  }
  *out = nc;
  return AMRVAC_OK;
}

int amrvac_set_path(amrvac_ctx* c, int path) {
  if (!c) return AMRVAC_E_ARG;
  if (path != AMRVAC_PATH_PLAIN && path != AMRVAC_PATH_FUSED) return fail(c, AMRVAC_E_ARG, "unknown path");
  if (path == AMRVAC_PATH_FUSED && c->G.nx != 16) return fail(c, AMRVAC_E_ARG, "the fused path needs block_nx = 16");
  if (path == AMRVAC_PATH_FUSED && c->G.ng != 2 && c->G.ng != 3)
    return fail(c, AMRVAC_E_ARG, "the fused path needs nghost = 2 or 3");
  if (path == AMRVAC_PATH_PLAIN && (c->g.precision != AMRVAC_FP64 || c->batch))
    return fail(c, AMRVAC_E_ARG, "the plain path is for single-job FP64 contexts");
  c->path = path;
  return AMRVAC_OK;
}

int amrvac_advance(amrvac_ctx* c, int nsteps, int nstages, int use_graph) {
  if (!c) return AMRVAC_E_ARG;
  if (c->batch) return fail(c, AMRVAC_E_STATE, "batch contexts step with amrvac_batch_step");
  if (nstages < 2 || nstages > 5) return fail(c, AMRVAC_E_ARG, "amrvac_advance supports 2 .. 5 stages");
  if ((int)c->slots.size() < slots_for_stages(nstages)) return fail(c, AMRVAC_E_ARG, "not enough slots");
  if (nsteps < 0) return fail(c, AMRVAC_E_ARG, "negative step count");
  if (int rc = ensure_tables(c)) return rc;
  if (int rc = ensure_plain_scratch(c)) return rc;
  double *dt = c->d_jdt, *ch = c->d_jch, *kap = c->d_jkappa;
  if (!use_graph) {
    for (int n = 0; n < nsteps; ++n)
      if (int rc = enqueue_step(c, nstages, dt, ch, kap)) return rc;
    return AMRVAC_OK;
  }
  // A captured step starts with the finalize-only cfl when its last stage
  // folds the CFL rate in; every replay then leaves the rate of slot 0 for
  // the next one.  Before the first replay the accumulators must hold it.
  if (can_carry(c) && c->carry_slot != 0) {
    drop_carry(c);
    if (int rc = clear_if_dirty(c)) return rc;
    HIP_TRY(c, launch_cfl_accumulate(c->stream, c->G, c->tables(), c->slots[0], c->P, c->d_status,
                                     cfl_state(c, dt, ch, kap)));
    c->carry_slot = 0;
  }
  if (!c->graph_exec || c->graph_stages != nstages || c->graph_path != c->path) {
    drop_graph(c);
    if (c->stream == nullptr) return fail(c, AMRVAC_E_STATE, "graph capture needs a non-null stream");
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_step(c, nstages, dt, ch, kap);
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &gr);
    if (rc) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    if (e != hipSuccess) return fail(c, AMRVAC_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    c->graph = gr;
    HIP_TRY(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
    c->graph_stages = nstages;
    c->graph_path = c->path;
  }
  for (int n = 0; n < nsteps; ++n) HIP_TRY(c, hipGraphLaunch(c->graph_exec, c->stream));
  return AMRVAC_OK;
}

int amrvac_set_tune(amrvac_ctx* c, const amrvac_tune* t) {
  if (!c) return AMRVAC_E_ARG;
  if (!t) return fail(c, AMRVAC_E_ARG, "null tune");
  if (t->zseg != 1 && t->zseg != 2 && t->zseg != 4) return fail(c, AMRVAC_E_ARG, "zseg must be 1, 2 or 4");
  if (c->G.ndim == 2 && t->zseg != 1) return fail(c, AMRVAC_E_ARG, "zseg must be 1 in 2D");
  if ((t->rotate != 0 && t->rotate != 1) || (t->xcd != 0 && t->xcd != 1))
    return fail(c, AMRVAC_E_ARG, "rotate and xcd are 0 or 1");
  const FusedTune nt{t->zseg, t->rotate, t->xcd};
  if (nt.zseg != c->tune.zseg || nt.rot != c->tune.rot || nt.xcd != c->tune.xcd) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    c->tune = nt;
  }
  return AMRVAC_OK;
}

int amrvac_get_tune(const amrvac_ctx* c, amrvac_tune* t) {
  if (!c || !t) return AMRVAC_E_ARG;
  t->zseg = c->tune.zseg;
  t->rotate = c->tune.rot;
  t->xcd = c->tune.xcd;
  return AMRVAC_OK;
}

int amrvac_autotune(amrvac_ctx* c, int in, int out, int reps, amrvac_tune* best, float* ms, int* ncand) {
  if (!c) return AMRVAC_E_ARG;
  if (c->batch) return fail(c, AMRVAC_E_STATE, "autotune a single-job context of the same shape");
  if (c->path != AMRVAC_PATH_FUSED) return fail(c, AMRVAC_E_STATE, "autotune needs the fused path");
  if (c->G.ng != 2) return fail(c, AMRVAC_E_STATE, "autotune tunes the fused stage of two ghost layers");
  if (int rc = check_slot(c, in)) return rc;
  if (int rc = check_slot(c, out)) return rc;
  if (in == out) return fail(c, AMRVAC_E_ARG, "in and out slots must differ");
  if (reps < 1 || reps > 1000) return fail(c, AMRVAC_E_ARG, "reps must be in 1..1000");
  if (int rc = ensure_tables(c)) return rc;
  // candidates, zseg-major then rotate then xcd
  std::vector<FusedTune> cand;
  for (int z : {1, 2, 4}) {
    if (c->G.ndim == 2 && z != 1) continue;
    for (int r = 0; r < 2; ++r)
      for (int x = 0; x < 2; ++x) cand.push_back(FusedTune{z, r, x});
  }
  // the status record (flags, fix count, last dt) is restored afterwards
  DevStatus* saved = nullptr;
  HIP_TRY(c, hipMalloc(&saved, sizeof(DevStatus)));
  std::vector<float> times(cand.size(), 0.0f);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMemcpyAsync(saved, c->d_status, sizeof(DevStatus), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int rc = AMRVAC_OK;
  if (e == hipSuccess) {
    drop_carry(c);
    touch_slot(c, out);
    rc = clear_if_dirty(c);
  }
  if (e == hipSuccess && rc == AMRVAC_OK)
    e = launch_cfl(c->stream, c->G, c->tables(), c->slots[in], c->P, c->d_status,
                   cfl_state(c, c->d_jdt, c->d_jch, c->d_jkappa));
  if (e == hipSuccess && rc == AMRVAC_OK) rc = fill_slot(c, in);
  const JobScalars J{c->d_jdt, c->d_jch, c->d_jkappa};
  const Tables T = c->tables();
  for (size_t k = 0; k < cand.size() && e == hipSuccess && rc == AMRVAC_OK; ++k) {
    e = launch_fused_stage(c->stream, c->G, T, J, cand[k], c->slots[in], c->slots[out], c->slots[out], 1.0, c->P,
                           c->d_status, nullptr, stage_freg(c));
    if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r)
      e = launch_fused_stage(c->stream, c->G, T, J, cand[k], c->slots[in], c->slots[out], c->slots[out], 1.0,
                             c->P, c->d_status, nullptr, stage_freg(c));
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&times[k], e0, e1);
    times[k] /= (float)reps;
  }
  if (e == hipSuccess && rc == AMRVAC_OK)
    e = hipMemcpyAsync(c->d_status, saved, sizeof(DevStatus), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && rc == AMRVAC_OK) e = hipStreamSynchronize(c->stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(saved);
  if (rc != AMRVAC_OK) return rc;
  if (e != hipSuccess) return fail(c, AMRVAC_E_HIP, std::string("autotune: ") + hipGetErrorString(e));
  size_t kb = 0;
  for (size_t k = 1; k < cand.size(); ++k)
    if (times[k] < times[kb]) kb = k;
  drop_graph(c);
  c->tune = cand[kb];
  if (best) amrvac_get_tune(c, best);
  if (ms)
    for (size_t k = 0; k < cand.size(); ++k) ms[k] = times[k];
  if (ncand) *ncand = (int)cand.size();
  return AMRVAC_OK;
}

int amrvac_sync_flags(amrvac_ctx* c, int* flags_host, long long* nfix_host, double* dt_host) {
  if (!c) return AMRVAC_E_ARG;
  DevStatus st{};
  HIP_TRY(c, hipMemcpyAsync(&st, c->d_status, sizeof(st), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (flags_host) *flags_host = (int)st.flags;
  if (nfix_host) *nfix_host = (long long)st.nfix;
  if (dt_host) *dt_host = st.last_dt;
  if ((st.flags & F_BAD_DT) || ((st.flags & (F_SMALL_RHO | F_SMALL_P)) && !c->g.fix_small_values))
    return fail(c, AMRVAC_E_NONPHYSICAL, "non-physical state (flags " + std::to_string(st.flags) + ")");
  return AMRVAC_OK;
}

int amrvac_reset_flags(amrvac_ctx* c) {
  if (!c) return AMRVAC_E_ARG;
  HIP_TRY(c, launch_reset_status(c->stream, c->d_status));
  return AMRVAC_OK;
}

// ---------------------------------------------------------------------------
// batch (serving) contexts

int amrvac_batch_create(amrvac_ctx** out, const amrvac_grid_desc* shape, int capacity_blocks, int max_jobs,
                        int nstages, void* const* slots, void* stream) {
  if (!out) return AMRVAC_E_ARG;
  *out = nullptr;
  std::string why;
  if (check_desc(shape, &why) != AMRVAC_OK) { g_init_err = why; return AMRVAC_E_ARG; }
  if (shape->block_nx != 16) {
    g_init_err = "batch contexts run the fused path: block_nx must be 16";
    return AMRVAC_E_ARG;
  }
  if (capacity_blocks < 1 || max_jobs < 1 || nstages < 2 || nstages > 5 || !slots) {
    g_init_err = "bad capacity, job count, stage count or slots";
    return AMRVAC_E_ARG;
  }
  const int nslots = slots_for_stages(nstages);
  for (int s = 0; s < nslots; ++s)
    if (!slots[s]) { g_init_err = "null slot pointer"; return AMRVAC_E_ARG; }
  amrvac_ctx* c = new amrvac_ctx();
  c->batch = true;
  c->batch_stages = nstages;
  c->cap = capacity_blocks;
  c->njob_cap = max_jobs;
  setup_shape(c, shape);
  c->path = AMRVAC_PATH_FUSED;
  c->stream = static_cast<hipStream_t>(stream);
  c->slots.clear();
  for (int k = 0; k < nslots; ++k) c->slots.push_back(static_cast<char*>(slots[k]) + slot_lead(shape->precision));
  (void)hipGetDevice(&c->device);
  c->jobs.resize(max_jobs);
  c->free_runs.push_back({0, capacity_blocks});
  int rc = alloc_context(c);
  if (!rc) rc = rebuild(c);
  if (rc) {
    g_init_err = c->err;
    free_all(c);
    delete c;
    return rc;
  }
  *out = c;
  return AMRVAC_OK;
}

int amrvac_batch_add_job(amrvac_ctx* c, const amrvac_grid_desc* g, int nb, const int* level, const int* ijk,
                         const double* prim_dev, int nsteps, int* job_out) {
  if (!c || !job_out) return AMRVAC_E_ARG;
  if (!c->batch) return fail(c, AMRVAC_E_STATE, "not a batch context");
  std::string why;
  if (check_desc(g, &why) != AMRVAC_OK) return fail(c, AMRVAC_E_ARG, why);
  const amrvac_grid_desc& s = c->g;
  if (g->ndim != s.ndim || g->block_nx != s.block_nx || g->nghost != s.nghost || g->precision != s.precision ||
      g->gamma != s.gamma ||
      g->small_density != s.small_density || g->small_pressure != s.small_pressure ||
      g->fix_small_values != s.fix_small_values || g->limiter != s.limiter || g->flux != s.flux ||
      std::memcmp(g->bc_fixed_prim, s.bc_fixed_prim, sizeof(s.bc_fixed_prim)) != 0)
    return fail(c, AMRVAC_E_ARG, "job shape or physics differs from the batch");
  if (nb < 1 || !level || !ijk || !prim_dev || nsteps < 0) return fail(c, AMRVAC_E_ARG, "bad job arguments");
  int jslot = -1;
  for (int j = 0; j < c->njob_cap; ++j)
    if (!c->jobs[j].used) {
      jslot = j;
      break;
    }
  if (jslot < 0) return fail(c, AMRVAC_E_NOMEM, "no free job slot");
  int run = -1;  // first fit in the free runs of the pool
  for (size_t r = 0; r < c->free_runs.size(); ++r)
    if (c->free_runs[r].second >= nb) {
      run = (int)r;
      break;
    }
  if (run < 0) return fail(c, AMRVAC_E_NOMEM, "no contiguous room for the job's blocks");
  const int first = c->free_runs[run].first;
  JobRec J;
  if (build_job(g, nb, level, ijk, first, &J.t) != AMRVAC_OK) return fail(c, AMRVAC_E_ARG, J.t.err);
  J.used = true;
  J.first = first;
  J.nb = nb;
  J.steps_left = nsteps;
  // (stream-ordered: kernels already queued still see the blocks' old tables)
  if (int rc = upload_job_blocks(c, J, jslot)) return rc;
  HIP_TRY(c, launch_set_prim(c->stream, c->G, first, nb, prim_dev, c->slots[0], c->P));
  c->free_runs[run].first += nb;
  c->free_runs[run].second -= nb;
  if (c->free_runs[run].second == 0) c->free_runs.erase(c->free_runs.begin() + run);
  c->jobs[jslot] = std::move(J);
  c->dirty = true;
  *job_out = jslot;
  return AMRVAC_OK;
}

int amrvac_batch_step(amrvac_ctx* c) {
  if (!c) return AMRVAC_E_ARG;
  if (!c->batch) return fail(c, AMRVAC_E_STATE, "not a batch context");
  if (int rc = ensure_tables(c)) return rc;
  if (c->n_order == 0) return AMRVAC_OK;
  if (int rc = ensure_plain_scratch(c)) return rc;
  if (int rc = enqueue_step(c, c->batch_stages, c->d_jdt, c->d_jch, c->d_jkappa)) return rc;
  for (int j = 0; j < c->njob_cap; ++j) {
    JobRec& J = c->jobs[j];
    if (J.used && J.steps_left > 0) {
      --J.steps_left;
      ++J.steps_done;
      if (J.steps_left == 0) c->dirty = true;
    }
  }
  return AMRVAC_OK;
}

int amrvac_batch_job_info(amrvac_ctx* c, int job, int* steps_done, int* steps_left, int* nblocks) {
  if (!c) return AMRVAC_E_ARG;
  if (!job_ok(c, job)) return fail(c, AMRVAC_E_ARG, "no such job");
  if (steps_done) *steps_done = c->jobs[job].steps_done;
  if (steps_left) *steps_left = c->jobs[job].steps_left;
  if (nblocks) *nblocks = c->jobs[job].nb;
  return AMRVAC_OK;
}

int amrvac_batch_get_job(amrvac_ctx* c, int job, double* cons_dev) {
  if (!c || !cons_dev) return AMRVAC_E_ARG;
  if (!job_ok(c, job)) return fail(c, AMRVAC_E_ARG, "no such job");
  const JobRec& J = c->jobs[job];
  HIP_TRY(c, launch_get_cons(c->stream, c->G, J.first, J.nb, c->slots[0], cons_dev));
  return AMRVAC_OK;
}

int amrvac_batch_remove_job(amrvac_ctx* c, int job) {
  if (!c) return AMRVAC_E_ARG;
  if (!job_ok(c, job)) return fail(c, AMRVAC_E_ARG, "no such job");
  JobRec& J = c->jobs[job];
  // host bookkeeping only: a later job placed in these blocks is written by
  // work queued behind everything already on the stream
  c->free_runs.push_back({J.first, J.nb});  // return the run, merging neighbours
  std::sort(c->free_runs.begin(), c->free_runs.end());
  std::vector<std::pair<int, int>> merged;
  for (const auto& r : c->free_runs) {
    if (!merged.empty() && merged.back().first + merged.back().second == r.first)
      merged.back().second += r.second;
    else
      merged.push_back(r);
  }
  c->free_runs.swap(merged);
  J = JobRec();
  c->dirty = true;
  return AMRVAC_OK;
}

int amrvac_batch_free_blocks(amrvac_ctx* c, int* largest_run, int* total_free) {
  if (!c) return AMRVAC_E_ARG;
  if (!c->batch) return fail(c, AMRVAC_E_STATE, "not a batch context");
  int big = 0, tot = 0;
  for (const auto& r : c->free_runs) {
    big = std::max(big, r.second);
    tot += r.second;
  }
  if (largest_run) *largest_run = big;
  if (total_free) *total_free = tot;
  return AMRVAC_OK;
}

}  // extern "C"
