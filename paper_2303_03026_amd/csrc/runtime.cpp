// Host runtime of the C ABI declared in include/amrvac.h: validates the block
// hierarchy, builds the face-neighbour and ghost-task tables, owns scratch
// memory and the per-step HIP graph, and enqueues the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/amrvac.h"
#include "kernels.h"

using namespace amrvac;

struct amrvac_ctx {
  amrvac_grid_desc g{};
  GridConst G{};
  LevelConst L{};
  PhysConst P{};
  FixedBC fixed{};
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<void*> slots;
  int path = AMRVAC_PATH_PLAIN;
  // device tables
  int* d_level = nullptr;
  int* d_pos = nullptr;
  int* d_link = nullptr;
  int* d_tasks_fill = nullptr;   // every copy/restrict/physical face (plain path)
  int n_tasks_fill = 0;
  int* d_tasks_fill_fused = nullptr;  // faces the fused stage does not read in place
  int n_tasks_fill_fused = 0;
  int* d_order = nullptr;  // Morton order of the blocks (fused stage scheduling)
  int* d_tasks_prolong = nullptr;
  int n_tasks_prolong = 0;
  int* d_tasks_reflux = nullptr;
  int n_tasks_reflux = 0;
  // scratch
  double* d_prim = nullptr;
  double* d_flux[3] = {nullptr, nullptr, nullptr};
  DevStatus* d_status = nullptr;
  double* d_scalars = nullptr;  // dt, c_h, kappa for amrvac_advance
  // graph of one step
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_stages = 0;
  int graph_path = -1;
  std::string err;
};

namespace {

struct KeyL {
  int l;
  long i, j, k;
  bool operator<(const KeyL& o) const { return std::tie(l, i, j, k) < std::tie(o.l, o.i, o.j, o.k); }
};

int fail(amrvac_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIP_TRY(ctx, expr)                                                            \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail((ctx), AMRVAC_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

thread_local std::string g_init_err;

int check_desc(const amrvac_grid_desc* g, std::string* why) {
  if (!g) { *why = "null descriptor"; return AMRVAC_E_ARG; }
  if (g->ndim != 2 && g->ndim != 3) { *why = "ndim must be 2 or 3"; return AMRVAC_E_ARG; }
  if (g->nghost != 2) { *why = "nghost must be 2 (van Leer stencil)"; return AMRVAC_E_ARG; }
  if (g->block_nx < 4 || g->block_nx > 16 || (g->block_nx & 1)) {
    *why = "block_nx must be even, 4..16";
    return AMRVAC_E_ARG;
  }
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
  return AMRVAC_OK;
}

long long slot_bytes_of(const amrvac_grid_desc* g, int nb) {
  const long pn = g->block_nx + 2 * g->nghost;
  const long pc = pn * pn * (g->ndim == 3 ? pn : 1);
  const long per = g->precision == AMRVAC_FP64 ? 72 : 40;
  return (long long)nb * pc * per;
}

static int free_all(amrvac_ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  void* ptrs[] = {c->d_level, c->d_pos, c->d_link, c->d_tasks_fill, c->d_tasks_fill_fused, c->d_order,
                  c->d_tasks_prolong, c->d_tasks_reflux,
                  c->d_prim, c->d_flux[0], c->d_flux[1], c->d_flux[2], c->d_status, c->d_scalars};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  return AMRVAC_OK;
}

template <class T>
static int upload(amrvac_ctx* c, T** dptr, const std::vector<T>& h) {
  const size_t n = std::max<size_t>(h.size(), 1) * sizeof(T);
  HIP_TRY(c, hipMalloc((void**)dptr, n));
  if (!h.empty()) HIP_TRY(c, hipMemcpy(*dptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return AMRVAC_OK;
}

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
  if (!out) return AMRVAC_E_ARG;
  *out = nullptr;
  std::string why;
  if (check_desc(g, &why) != AMRVAC_OK) { g_init_err = why; return AMRVAC_E_ARG; }
  if (g->precision != AMRVAC_FP64) { g_init_err = "FP32-mixed storage is not available in this build"; return AMRVAC_E_ARG; }
  if (nb < 1 || !level || !ijk || !slots || nslots < 1) { g_init_err = "need blocks, tables and slots"; return AMRVAC_E_ARG; }
  for (int s = 0; s < nslots; ++s)
    if (!slots[s]) { g_init_err = "null slot pointer"; return AMRVAC_E_ARG; }

  const int ndim = g->ndim, nx = g->block_nx;
  // ---- block set validation -------------------------------------------------
  std::map<KeyL, int> leaf;
  std::set<KeyL> refined;
  int finest = 1;
  double vol = 0.0;
  for (int b = 0; b < nb; ++b) {
    const int l = level[b];
    if (l < 1 || l > MAXLEV) { g_init_err = "level out of range 1..12"; return AMRVAC_E_ARG; }
    long p[3] = {ijk[3 * b], ijk[3 * b + 1], ndim == 3 ? ijk[3 * b + 2] : 0};
    for (int d = 0; d < ndim; ++d)
      if (p[d] < 0 || p[d] >= ((long)g->base_blocks[d] << (l - 1))) { g_init_err = "block outside the domain"; return AMRVAC_E_ARG; }
    if (!leaf.emplace(KeyL{l, p[0], p[1], p[2]}, b).second) { g_init_err = "duplicate block"; return AMRVAC_E_ARG; }
    finest = std::max(finest, l);
    vol += std::ldexp(1.0, -ndim * (l - 1));
    for (int m = l - 1; m >= 1; --m) {
      for (int d = 0; d < 3; ++d) p[d] >>= 1;
      refined.insert(KeyL{m, p[0], p[1], p[2]});
    }
  }
  for (const auto& kv : leaf)
    if (refined.count(kv.first)) { g_init_err = "blocks overlap (a leaf is also refined)"; return AMRVAC_E_ARG; }
  const double nbase = (double)g->base_blocks[0] * g->base_blocks[1] * (ndim == 3 ? g->base_blocks[2] : 1);
  if (std::fabs(vol - nbase) > 1e-9 * nbase) { g_init_err = "blocks do not tile the domain"; return AMRVAC_E_ARG; }

  auto nblk = [&](int l, int d) -> long { return d < ndim ? ((long)g->base_blocks[d] << (l - 1)) : 1; };
  auto periodic = [&](int d) { return g->bc_lo[d] == AMRVAC_BC_PERIODIC; };
  // 2:1 nesting over faces, edges and corners: every slot next to a leaf of
  // level l is a leaf, refined, or inside a leaf of level l-1.
  for (const auto& kv : leaf) {
    const int l = kv.first.l;
    const long p[3] = {kv.first.i, kv.first.j, kv.first.k};
    for (int oz = (ndim == 3 ? -1 : 0); oz <= (ndim == 3 ? 1 : 0); ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          long q[3] = {p[0] + ox, p[1] + oy, p[2] + oz};
          bool skip = false;
          for (int d = 0; d < ndim; ++d) {
            if (q[d] < 0 || q[d] >= nblk(l, d)) {
              if (periodic(d)) q[d] = (q[d] + nblk(l, d)) % nblk(l, d);
              else skip = true;
            }
          }
          if (skip) continue;
          const KeyL k{l, q[0], q[1], q[2]};
          if (leaf.count(k)) continue;
          if (refined.count(k)) {
            // children facing this leaf must be leaves (not refined further)
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
                  if (!leaf.count(ck)) { g_init_err = "hierarchy is not 2:1 nested (finer by two)"; return AMRVAC_E_ARG; }
                }
            continue;
          }
          if (l >= 2 && leaf.count(KeyL{l - 1, q[0] >> 1, q[1] >> 1, ndim == 3 ? q[2] >> 1 : 0})) continue;
          g_init_err = "hierarchy is not 2:1 nested (coarser by two)";
          return AMRVAC_E_ARG;
        }
  }

  amrvac_ctx* c = new amrvac_ctx();
  c->g = *g;
  c->stream = static_cast<hipStream_t>(stream);
  c->slots.assign(slots, slots + nslots);
  (void)hipGetDevice(&c->device);
  GridConst& G = c->G;
  G.ndim = ndim;
  G.nx = nx;
  G.ng = g->nghost;
  G.pn = nx + 2 * G.ng;
  G.nb = nb;
  G.nfaces = (nx + 1) * nx * (ndim == 3 ? nx : 1);
  G.pcells = (long)G.pn * G.pn * (ndim == 3 ? G.pn : 1);
  G.icells = (long)nx * nx * (ndim == 3 ? nx : 1);
  for (int d = 0; d < 3; ++d) G.base[d] = d < ndim ? g->base_blocks[d] : 1;
  G.precision = g->precision;

  LevelConst& L = c->L;
  for (int l = 1; l <= MAXLEV; ++l)
    for (int d = 0; d < 3; ++d) {
      const double dx = d < ndim ? (g->xmax[d] - g->xmin[d]) / (double)(nblk(l, d) * nx) : 1.0;
      L.dx[l][d] = dx;
      L.inv_dx[l][d] = 1.0 / dx;
    }
  L.sum_inv_dx_fin = 0.0;
  L.min_dx_fin = L.dx[finest][0];
  for (int d = 0; d < ndim; ++d) {
    L.sum_inv_dx_fin += 1.0 / L.dx[finest][d];
    L.min_dx_fin = std::min(L.min_dx_fin, L.dx[finest][d]);
  }
  L.cfl = g->cfl;
  L.glm_alpha = g->glm_alpha;
  c->P = PhysConst{g->gamma, g->gamma - 1.0, 1.0 / (g->gamma - 1.0), g->small_density, g->small_pressure,
                   g->fix_small_values};
  std::memcpy(c->fixed.prim, g->bc_fixed_prim, sizeof(c->fixed.prim));

  // ---- face links and task lists -------------------------------------------
  std::vector<int> link((size_t)nb * 6 * LINK_INTS, -1), pos((size_t)nb * 3), lev(nb);
  std::vector<int> tfill, tprol, trefl;
  for (int b = 0; b < nb; ++b) {
    const int l = level[b];
    lev[b] = l;
    const long p[3] = {ijk[3 * b], ijk[3 * b + 1], ndim == 3 ? ijk[3 * b + 2] : 0};
    for (int d = 0; d < 3; ++d) pos[3 * b + d] = (int)p[d];
    for (int d = 0; d < ndim; ++d)
      for (int side = 0; side < 2; ++side) {
        int* Lk = &link[((size_t)b * 6 + d * 2 + side) * LINK_INTS];
        long q[3] = {p[0], p[1], p[2]};
        q[d] += side ? 1 : -1;
        if (q[d] < 0 || q[d] >= nblk(l, d)) {
          if (!periodic(d)) {
            Lk[0] = LINK_PHYS;
            Lk[1] = side ? g->bc_hi[d] : g->bc_lo[d];
            tfill.push_back(b);
            tfill.push_back(d * 2 + side);
            continue;
          }
          q[d] = (q[d] + nblk(l, d)) % nblk(l, d);
        }
        auto it = leaf.find(KeyL{l, q[0], q[1], q[2]});
        if (it != leaf.end()) {
          Lk[0] = LINK_SAME;
          Lk[1] = it->second;
          tfill.push_back(b);
          tfill.push_back(d * 2 + side);
          continue;
        }
        if (refined.count(KeyL{l, q[0], q[1], q[2]})) {
          Lk[0] = LINK_FINE;
          const int ta = d == 0 ? 1 : 0, tb = d == 2 ? 1 : 2;
          for (int ob = 0; ob < (ndim == 3 ? 2 : 1); ++ob)
            for (int oa = 0; oa < 2; ++oa) {
              long cq[3] = {2 * q[0], 2 * q[1], ndim == 3 ? 2 * q[2] : 0};
              cq[d] += side ? 0 : 1;
              cq[ta] += oa;
              if (ndim == 3) cq[tb] += ob;
              auto ci = leaf.find(KeyL{l + 1, cq[0], cq[1], cq[2]});
              if (ci == leaf.end()) {
                delete c;
                g_init_err = "fine neighbour is not a leaf";
                return AMRVAC_E_ARG;
              }
              Lk[1 + ob * 2 + oa] = ci->second;
            }
          tfill.push_back(b);
          tfill.push_back(d * 2 + side);
          trefl.push_back(b);
          trefl.push_back(d * 2 + side);
          continue;
        }
        auto pi = leaf.find(KeyL{l - 1, q[0] >> 1, q[1] >> 1, ndim == 3 ? q[2] >> 1 : 0});
        if (l < 2 || pi == leaf.end()) {
          delete c;
          g_init_err = "face neighbour not found (hierarchy not 2:1 nested)";
          return AMRVAC_E_ARG;
        }
        Lk[0] = LINK_COARSE;
        Lk[1] = pi->second;
        Lk[2] = l;
        tprol.push_back(b);
        tprol.push_back(d * 2 + side);
      }
  }
  c->n_tasks_fill = (int)tfill.size() / 2;
  c->n_tasks_prolong = (int)tprol.size() / 2;
  c->n_tasks_reflux = g->reflux ? (int)trefl.size() / 2 : 0;
  // The fused stage reads same-level neighbours in place; it needs filled
  // ghosts only on faces towards finer leaves and physical boundaries, plus
  // every face of a block whose ghosts feed a prolongation.
  std::vector<char> prol_src(nb, 0);
  for (size_t q = 0; q < tprol.size(); q += 2) {
    const int fb = tprol[q], face = tprol[q + 1];
    prol_src[link[((size_t)fb * 6 + face) * LINK_INTS + 1]] = 1;
  }
  std::vector<int> tfused;
  for (size_t q = 0; q < tfill.size(); q += 2) {
    const int fb = tfill[q], face = tfill[q + 1];
    if (link[((size_t)fb * 6 + face) * LINK_INTS] != LINK_SAME || prol_src[fb]) {
      tfused.push_back(fb);
      tfused.push_back(face);
    }
  }
  c->n_tasks_fill_fused = (int)tfused.size() / 2;
  // Morton order on the finest level's block grid
  std::vector<std::pair<unsigned long long, int>> keyed(nb);
  for (int b = 0; b < nb; ++b) {
    const int sft = finest - level[b];
    unsigned long long key = 0;
    const unsigned long long q0 = (unsigned long long)pos[3 * b] << sft, q1 = (unsigned long long)pos[3 * b + 1] << sft,
                             q2 = (unsigned long long)pos[3 * b + 2] << sft;
    for (int bit = 0; bit < 20; ++bit) {
      key |= ((q0 >> bit) & 1ull) << (3 * bit);
      key |= ((q1 >> bit) & 1ull) << (3 * bit + 1);
      key |= ((q2 >> bit) & 1ull) << (3 * bit + 2);
    }
    keyed[b] = {key, b};
  }
  std::sort(keyed.begin(), keyed.end());
  std::vector<int> order(nb);
  for (int b = 0; b < nb; ++b) order[b] = keyed[b].second;

  int rc;
  if ((rc = upload(c, &c->d_level, lev)) || (rc = upload(c, &c->d_pos, pos)) || (rc = upload(c, &c->d_link, link)) ||
      (rc = upload(c, &c->d_tasks_fill, tfill)) || (rc = upload(c, &c->d_tasks_prolong, tprol)) ||
      (rc = upload(c, &c->d_tasks_fill_fused, tfused)) || (rc = upload(c, &c->d_order, order)) ||
      (rc = upload(c, &c->d_tasks_reflux, trefl))) {
    g_init_err = c->err;
    free_all(c);
    delete c;
    return rc;
  }
  auto alloc = [&](void** p, size_t n) -> int {
    hipError_t e = hipMalloc(p, n);
    if (e != hipSuccess) {
      g_init_err = std::string("hipMalloc of library scratch failed: ") + hipGetErrorString(e);
      return AMRVAC_E_NOMEM;
    }
    return AMRVAC_OK;
  };
  if ((rc = alloc((void**)&c->d_prim, (size_t)nb * NV * G.pcells * sizeof(double))) ||
      (rc = alloc((void**)&c->d_flux[0], (size_t)nb * NV * G.nfaces * sizeof(double))) ||
      (rc = alloc((void**)&c->d_flux[1], (size_t)nb * NV * G.nfaces * sizeof(double))) ||
      (ndim == 3 && (rc = alloc((void**)&c->d_flux[2], (size_t)nb * NV * G.nfaces * sizeof(double)))) ||
      (rc = alloc((void**)&c->d_status, sizeof(DevStatus))) ||
      (rc = alloc((void**)&c->d_scalars, 4 * sizeof(double)))) {
    free_all(c);
    delete c;
    return rc;
  }
  hipError_t e = hipMemset(c->d_status, 0, sizeof(DevStatus));
  if (e == hipSuccess) e = hipMemset(c->d_scalars, 0, 4 * sizeof(double));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    g_init_err = std::string("init: ") + hipGetErrorString(e);
    free_all(c);
    delete c;
    return AMRVAC_E_HIP;
  }
  *out = c;
  return AMRVAC_OK;
}

static int check_slot(amrvac_ctx* c, int s) {
  if (s < 0 || s >= (int)c->slots.size()) return fail(c, AMRVAC_E_ARG, "slot index out of range");
  return AMRVAC_OK;
}

int amrvac_set_primitive(amrvac_ctx* c, int slot, const double* prim_dev) {
  if (!c) return AMRVAC_E_ARG;
  if (int rc = check_slot(c, slot)) return rc;
  if (!prim_dev) return fail(c, AMRVAC_E_ARG, "null primitive array");
  HIP_TRY(c, launch_set_prim(c->stream, c->G, prim_dev, c->slots[slot], c->P));
  return AMRVAC_OK;
}

int amrvac_get_conserved(amrvac_ctx* c, int slot, double* cons_dev) {
  if (!c) return AMRVAC_E_ARG;
  if (int rc = check_slot(c, slot)) return rc;
  if (!cons_dev) return fail(c, AMRVAC_E_ARG, "null output array");
  HIP_TRY(c, launch_get_cons(c->stream, c->G, c->slots[slot], cons_dev));
  return AMRVAC_OK;
}

int amrvac_fill_ghosts(amrvac_ctx* c, int slot) {
  if (!c) return AMRVAC_E_ARG;
  if (int rc = check_slot(c, slot)) return rc;
  const bool fused = c->path == AMRVAC_PATH_FUSED;
  HIP_TRY(c, launch_fill_faces(c->stream, c->G, fused ? c->d_tasks_fill_fused : c->d_tasks_fill,
                               fused ? c->n_tasks_fill_fused : c->n_tasks_fill, c->d_link, c->d_pos,
                               c->slots[slot], c->P, c->fixed));
  HIP_TRY(c, launch_fill_faces(c->stream, c->G, c->d_tasks_prolong, c->n_tasks_prolong, c->d_link, c->d_pos,
                               c->slots[slot], c->P, c->fixed));
  return AMRVAC_OK;
}

int amrvac_cfl_dt(amrvac_ctx* c, int slot, double* dt_dev, double* ch_dev, double* kappa_dev) {
  if (!c) return AMRVAC_E_ARG;
  if (int rc = check_slot(c, slot)) return rc;
  if (!dt_dev || !ch_dev || !kappa_dev) return fail(c, AMRVAC_E_ARG, "null dt/c_h/kappa pointer");
  HIP_TRY(c, launch_cfl(c->stream, c->G, c->L, c->d_level, c->slots[slot], c->P, c->d_status, dt_dev, ch_dev,
                        kappa_dev));
  return AMRVAC_OK;
}

static int stage_plain(amrvac_ctx* c, int in, int base, int out, double w, const double* dt_dev,
                       const double* ch_dev, const double* kappa_dev) {
  HIP_TRY(c, launch_prim(c->stream, c->G, c->slots[in], c->d_prim, c->P, c->d_status));
  for (int d = 0; d < c->G.ndim; ++d)
    HIP_TRY(c, launch_flux(c->stream, c->G, d, c->d_prim, c->d_flux[d], ch_dev, c->P));
  FluxPtrs fp{{c->d_flux[0], c->d_flux[1], c->d_flux[2]}};
  HIP_TRY(c, launch_reflux(c->stream, c->G, c->d_tasks_reflux, c->n_tasks_reflux, c->d_link, fp));
  HIP_TRY(c, launch_update(c->stream, c->G, c->L, c->d_level, c->slots[in], c->slots[base], c->slots[out], w, fp,
                           dt_dev, kappa_dev));
  return AMRVAC_OK;
}

static int stage_fused(amrvac_ctx* c, int in, int base, int out, double w, const double* dt_dev,
                       const double* ch_dev, const double* kappa_dev) {
  HIP_TRY(c, launch_fused_stage(c->stream, c->G, c->L, c->d_level, c->d_link, c->d_order, c->slots[in],
                                c->slots[base], c->slots[out], w, dt_dev, ch_dev, kappa_dev, c->P, c->d_status));
  HIP_TRY(c, launch_reflux_correct(c->stream, c->G, c->L, c->d_level, c->d_tasks_reflux, c->n_tasks_reflux,
                                   c->d_link, c->slots[in], c->slots[out], w, dt_dev, ch_dev, c->P));
  return AMRVAC_OK;
}

int amrvac_stage(amrvac_ctx* c, int in, int base, int out, double w, const double* dt_dev, const double* ch_dev,
                 const double* kappa_dev) {
  if (!c) return AMRVAC_E_ARG;
  if (int rc = check_slot(c, in)) return rc;
  if (int rc = check_slot(c, out)) return rc;
  if (w != 1.0) {
    if (int rc = check_slot(c, base)) return rc;
  } else {
    base = out;
  }
  if (in == out) return fail(c, AMRVAC_E_ARG, "in and out slots must differ");
  if (base == in && w != 1.0) return fail(c, AMRVAC_E_ARG, "base must differ from in");
  if (!dt_dev || !ch_dev || !kappa_dev) return fail(c, AMRVAC_E_ARG, "null dt/c_h/kappa pointer");
  if (!(w > 0.0 && w <= 1.0)) return fail(c, AMRVAC_E_ARG, "stage weight must be in (0, 1]");
  if (c->path == AMRVAC_PATH_FUSED) return stage_fused(c, in, base, out, w, dt_dev, ch_dev, kappa_dev);
  return stage_plain(c, in, base, out, w, dt_dev, ch_dev, kappa_dev);
}

int amrvac_set_path(amrvac_ctx* c, int path) {
  if (!c) return AMRVAC_E_ARG;
  if (path != AMRVAC_PATH_PLAIN && path != AMRVAC_PATH_FUSED) return fail(c, AMRVAC_E_ARG, "unknown path");
  if (path == AMRVAC_PATH_FUSED && c->G.nx != 16) return fail(c, AMRVAC_E_ARG, "the fused path needs block_nx = 16");
  c->path = path;
  return AMRVAC_OK;
}

static int enqueue_step(amrvac_ctx* c, int nstages) {
  double* dt = c->d_scalars;
  double* ch = c->d_scalars + 1;
  double* kap = c->d_scalars + 2;
  int rc;
  if ((rc = amrvac_cfl_dt(c, 0, dt, ch, kap))) return rc;
  if (nstages == 2) {
    if ((rc = amrvac_fill_ghosts(c, 0)) || (rc = amrvac_stage(c, 0, 0, 1, 1.0, dt, ch, kap))) return rc;
    if ((rc = amrvac_fill_ghosts(c, 1)) || (rc = amrvac_stage(c, 1, 0, 0, 0.5, dt, ch, kap))) return rc;
    return AMRVAC_OK;
  }
  if ((rc = amrvac_fill_ghosts(c, 0)) || (rc = amrvac_stage(c, 0, 0, 1, 1.0, dt, ch, kap))) return rc;
  if ((rc = amrvac_fill_ghosts(c, 1)) || (rc = amrvac_stage(c, 1, 0, 2, 0.25, dt, ch, kap))) return rc;
  if ((rc = amrvac_fill_ghosts(c, 2)) || (rc = amrvac_stage(c, 2, 0, 0, 2.0 / 3.0, dt, ch, kap))) return rc;
  return AMRVAC_OK;
}

int amrvac_advance(amrvac_ctx* c, int nsteps, int nstages, int use_graph) {
  if (!c) return AMRVAC_E_ARG;
  if (nstages != 2 && nstages != 3) return fail(c, AMRVAC_E_ARG, "amrvac_advance supports 2 or 3 stages");
  if ((int)c->slots.size() < (nstages == 3 ? 3 : 2)) return fail(c, AMRVAC_E_ARG, "not enough slots");
  if (nsteps < 0) return fail(c, AMRVAC_E_ARG, "negative step count");
  if (!use_graph) {
    for (int n = 0; n < nsteps; ++n)
      if (int rc = enqueue_step(c, nstages)) return rc;
    return AMRVAC_OK;
  }
  if (!c->graph_exec || c->graph_stages != nstages || c->graph_path != c->path) {
    if (c->graph_exec) {
      (void)hipGraphExecDestroy(c->graph_exec);
      c->graph_exec = nullptr;
    }
    if (c->graph) {
      (void)hipGraphDestroy(c->graph);
      c->graph = nullptr;
    }
    if (c->stream == nullptr) return fail(c, AMRVAC_E_STATE, "graph capture needs a non-null stream");
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_step(c, nstages);
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

}  // extern "C"
