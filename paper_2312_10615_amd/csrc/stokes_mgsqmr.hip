// MG-SQMR driver and C ABI (include/stokes_mgsqmr.h) for gfx950.
//
// Host code sequences the kernels of kernels.hpp on the caller's stream:
//   V-cycle (Alg. 1) -> SMOOTH (Alg. 3) -> symmetric Vanka / symmetric DGS
//   SQMR (Alg. 4)    -> operator apply + fused reductions, BLAS-1 updates
// The SQMR scalars are reduced on the device in a fixed order and read back
// once per reduction, so results are bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/stokes_mgsqmr.h"
#include "host_tables.hpp"
#include "packed_kernels.hpp"
#include "kernels.hpp"

using namespace sg;

namespace {

// Level buffers hold the V-cycle's storage type (double, or float for an
// FP32 V-cycle).
struct Level {
  Geom g;
  void* b = nullptr;     // right-hand side (levels >= 1; level 0 only for an FP32 V-cycle)
  void* x = nullptr;     // iterate (same)
  void* r = nullptr;     // residual scratch (all but the coarsest)
  void* dscr = nullptr;  // DGS pressure-step deltas (p field)
  int* vcells[27] = {};   // V1 cells per colour class (8 or 27 classes)
  int nv[27] = {};
  long doff[27] = {};     // class slice of the Vanka delta buffer (additive Vanka keeps all classes)
  void* kinv = nullptr;  // Vanka local inverses, 8 x 8 per type (64 types for a box)
  void* alt = nullptr;   // second copy of the state for the two-copy Vanka passes (k_vanka_pp*)
  bool pp = false;       // this level runs them
  void* xs = nullptr;    // x-slab of the one-thread-per-subdomain Vanka passes (k_vanka_*_xs)
  bool sweep_ok = true;  // the one-workgroup Vanka step may run here (its LDS holds 64 types)
  uint32_t* flags = nullptr;  // labelled domain: the level's flag words (device)
};

struct Carver {
  char* base;
  size_t used = 0, cap;
  bool dry;
  Carver(void* b, size_t c, bool d) : base((char*)b), cap(c), dry(d) {}
  template <typename T>
  T* take(size_t count) {
    used = (used + 255) & ~size_t(255);
    T* p = dry ? nullptr : (T*)(base + used);
    used += count * sizeof(T);
    return p;
  }
};

}  // namespace

struct stokes_ctx {
  stokes_params prm{};
  int L = 0;
  std::vector<Level> lev;
  hipStream_t stream = nullptr;   // the caller's stream: everything runs here
  hipStream_t ks = nullptr;       // stream the V-cycle launches go to (= stream, or cap while capturing)
  hipStream_t cap = nullptr;      // private stream used only to capture V-cycle graphs
  long total = 0;  // elements of a finest-level state vector
  // SQMR vectors
  double *s = nullptr, *t = nullptr, *q = nullptr, *d = nullptr;
  // reductions
  double* partial = nullptr;
  int npartial = 0;
  double* dscal = nullptr;   // device scalars: reduction results
  double* hscal = nullptr;   // host mirror: pinned, or hscal_local for a context on the static scratch
  double hscal_local[16] = {};
  bool on_static = false;    // workspace = the library's static scratch (stokes_solve_static)
  // coarsest level
  double* cinv = nullptr;
  int* cdof = nullptr;
  int nc = 0;
  // Vanka delta scratch (max colour count x 8)
  void* vdelta = nullptr;
  int prec = 64;  // V-cycle precision
  // labelled domain (stokes_params.labels): per-level labels and host tables
  bool labelled = false;
  bool neumann = false;           // some unknown face borders an exterior cell: pressure is unique
  std::vector<Labels> labs;
  std::vector<LevelLabels> ll;
  // kernel timing (diagnostics)
  int prof_class = STOKES_KC_OFF, prof_level = -1;
  struct Pending { int k, l; hipEvent_t a, b; };
  // V-cycle graphs, keyed by input/output pointers and the profiling selection:
  // a sequence of graph segments and eagerly launched (timed) kernels
  struct Step {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::function<void()> fn;
    int k = -1, l = -1;
  };
  struct GraphEntry {
    const double* s;
    double* t;
    int pc, pl;
    int io;  // PC_* flags the V-cycle was captured with
    std::vector<Step> steps;
  };
  std::vector<GraphEntry> graphs;
  std::vector<Step> steps;      // segments of the graph being captured
  bool capturing = false;
  hipError_t cap_error = hipSuccess;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::vector<double> prof_ms;     // [class * 32 + level]
  std::vector<long> prof_n;
  bool prof_on(int k, int l) const {
    return prof_class != STOKES_KC_OFF && (prof_class == STOKES_KC_ALL || prof_class == k) &&
           (prof_level < 0 || prof_level == l);
  }
  hipEvent_t event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

namespace {

// Records HIP events around one launch when that kernel class/level is selected.
struct Prof {
  stokes_ctx* c;
  int k, l;
  hipEvent_t a = nullptr;
  Prof(stokes_ctx* c_, int k_, int l_) : c(c_), k(k_), l(l_) {
    if (c->prof_on(k, l)) {
      a = c->event();
      if (a) (void)hipEventRecord(a, c->ks);
    }
  }
  ~Prof() {
    if (!a) return;
    hipEvent_t b = c->event();
    if (!b) {
      c->pool.push_back(a);
      return;
    }
    (void)hipEventRecord(b, c->ks);
    c->pending.push_back({k, l, a, b});
  }
};

// Fold finished event pairs into the accumulators (waits for them).
void prof_collect(stokes_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      const int slot = p.k * 32 + (p.l < 32 ? p.l : 31);
      c->prof_ms[slot] += ms;
      c->prof_n[slot] += 1;
    }
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
}

void drop_graphs(stokes_ctx* c) {
  for (auto& e : c->graphs)
    for (auto& st : e.steps) {
      if (st.exec) (void)hipGraphExecDestroy(st.exec);
      if (st.graph) (void)hipGraphDestroy(st.graph);
    }
  c->graphs.clear();
}

int grid_for(long slots) {
  long nb = (slots + BS - 1) / BS;
  nb = (nb + NXCD - 1) / NXCD * NXCD;
  return (int)nb;
}

// Cells per thread of the packed kernels: one 16-byte load per operand.
template <typename T>
constexpr int dgs_pack() {
  return 16 / (int)sizeof(T);
}

template <typename T>
int apply_grid(const Geom& g) {  // k_apply_v: slot packs of each row
  return slab_blocks(g, slot_packs_per_row<dgs_pack<T>()>(g));
}

template <typename T>
int dgs_grid(const Geom& g) {  // packed DGS kernels: packs of one colour per row
  return slab_blocks(g, pack_per_row<dgs_pack<T>()>(g));
}

int restrict_grid(const Geom& gc) { return slab_blocks(gc, gc.sy); }  // k_restrict: one item per coarse slot
int prolong_grid(const Geom& gc) { return slab_blocks(gc, (gc.nx + 1) >> 1); }  // k_prolong_pairs: one per pair of coarse cells
int prolong_edge_grid(const Geom& g) {  // k_prolong_edge: one per face of the three last face planes
  const long n = (long)g.ny * g.nz + (long)g.nx * g.nz + (long)g.nx * g.ny;
  return (int)((n + BS - 1) / BS);
}

#define HIPCHK(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return STOKES_EDEVICE;      \
  } while (0)

int vanka_classes(const stokes_params& p) { return p.vanka == STOKES_VANKA_MULT27 ? 27 : 8; }

// Levels whose Vanka step runs in one workgroup (k_vanka_sweep).
bool vsweep_level(const Level& lv, int nc) {
  if (!lv.sweep_ok) return false;
  for (int k = 0; k < nc; ++k)
    if (lv.nv[k] > VSWEEP_MAX_CLASS) return false;
  return true;
}

long coarse_dofs(const Geom& g) {
  return (long)(g.nx - 1) * g.ny * g.nz + (long)g.nx * (g.ny - 1) * g.nz + (long)g.nx * g.ny * (g.nz - 1) +
         (long)g.nx * g.ny * g.nz;
}

int validate(const stokes_params* p, int* levels_out) {
  if (!p) return STOKES_EINVAL;
  if (p->nx < 2 || p->ny < 2 || p->nz < 2) return STOKES_EINVAL;
  if (!(p->h > 0) || !(p->eta > 0) || !(p->gamma > 0) || !std::isfinite(p->h) || !std::isfinite(p->eta) ||
      !std::isfinite(p->gamma))
    return STOKES_EINVAL;
  if (p->nu < 1 || p->n_boundary < 1) return STOKES_EINVAL;
  if (p->smoother != STOKES_SMOOTHER_SPLIT && p->smoother != STOKES_SMOOTHER_SYMMETRIC) return STOKES_EINVAL;
  if (p->smoother == STOKES_SMOOTHER_SYMMETRIC && (p->nu % 2)) return STOKES_EINVAL;
  if (p->vcycle_precision != 64 && p->vcycle_precision != 32) return STOKES_EINVAL;
  if (p->vanka != STOKES_VANKA_MULT8 && p->vanka != STOKES_VANKA_MULT27 && p->vanka != STOKES_VANKA_ADDITIVE)
    return STOKES_EINVAL;
  if (p->cycle != 1 && p->cycle != 2) return STOKES_EINVAL;
  if (p->labels) {  // Section 5 labels: values 0..2, no interior cell on the outer layer, some interior cell
    long interior = 0;
    for (int k = 0; k < p->nz + 2; ++k)
      for (int j = 0; j < p->ny + 2; ++j)
        for (int i = 0; i < p->nx + 2; ++i) {
          const uint8_t v = p->labels[i + (long)(p->nx + 2) * (j + (long)(p->ny + 2) * k)];
          if (v > CELL_EXTERIOR) return STOKES_EINVAL;
          const bool outer = i == 0 || j == 0 || k == 0 || i == p->nx + 1 || j == p->ny + 1 || k == p->nz + 1;
          if (v == CELL_INTERIOR && outer) return STOKES_EINVAL;
          interior += v == CELL_INTERIOR;
        }
    if (interior == 0) return STOKES_EINVAL;
  }
  int L = p->levels;
  if (L == 0) L = count_levels(p->nx, p->ny, p->nz, 4);
  if (L < 1 || L > count_levels(p->nx, p->ny, p->nz, 2)) return STOKES_EINVAL;
  // 32-bit slot arithmetic inside the kernels
  Geom g0 = make_geom(p->nx, p->ny, p->nz, p->h, p->eta, p->gamma, 0);
  if ((long)g0.field * 4 >= (1L << 31) - 1024) return STOKES_EINVAL;
  // dense coarsest solve: keep its inverse modest
  Geom gc = make_geom(p->nx, p->ny, p->nz, p->h, p->eta, p->gamma, L - 1);
  if (coarse_dofs(gc) > 2500) return STOKES_EINVAL;
  *levels_out = L;
  return STOKES_OK;
}

// Lay out (or size, when dry) everything the context keeps in the workspace.
void carve(stokes_ctx* c, Carver& cv, int L) {
  const stokes_params& p = c->prm;
  c->prec = p.vcycle_precision;
  const size_t es = c->prec == 32 ? sizeof(float) : sizeof(double);
  c->lev.assign(L, Level{});
  for (int l = 0; l < L; ++l) c->lev[l].g = make_geom(p.nx, p.ny, p.nz, p.h, p.eta, p.gamma, l);
  c->labelled = p.labels != nullptr;
  if (c->labelled && (int)c->ll.size() != L) {
    c->labs.assign(L, Labels{});
    c->ll.assign(L, LevelLabels{});
    Labels& l0 = c->labs[0];
    l0.nx = p.nx;
    l0.ny = p.ny;
    l0.nz = p.nz;
    l0.v.assign(p.labels, p.labels + (size_t)(p.nx + 2) * (p.ny + 2) * (p.nz + 2));
    for (int l = 0; l < L; ++l) {
      if (l > 0) c->labs[l] = coarsen(c->labs[l - 1]);
      label_tables(c->lev[l].g, c->labs[l], c->ll[l]);
    }
    c->neumann = c->ll[0].neumann;
  }
  const Geom& g0 = c->lev[0].g;
  c->total = 4L * g0.field;
  c->s = cv.take<double>(c->total);
  c->t = cv.take<double>(c->total);
  c->q = cv.take<double>(c->total);
  c->d = cv.take<double>(c->total);
  long maxblk = RED_BLOCKS;
  for (int l = 0; l < L; ++l)
    maxblk = std::max<long>(maxblk, std::max(grid_for(c->lev[l].g.field), apply_grid<double>(c->lev[l].g)));
  c->npartial = (int)maxblk;
  c->partial = cv.take<double>(2 * maxblk);
  c->dscal = cv.take<double>(16);
  long vmax = 0;
  for (int l = 0; l < L; ++l) {
    Level& lv = c->lev[l];
    const long tot = 4L * lv.g.field;
    if (l > 0 || c->prec == 32) {
      lv.b = cv.take<char>(tot * es);
      lv.x = cv.take<char>(tot * es);
    }
    if (c->labelled) lv.flags = cv.take<uint32_t>(lv.g.field);
    if (l < L - 1) {
      // residual scratch, also the plane sums of k_resid_restrict_xy
      lv.r = cv.take<char>(std::max<long>(tot, rr_elems(lv.g, c->lev[l + 1].g)) * es);
      lv.dscr = cv.take<char>(lv.g.field * es);
      // at least 64 types: the one-workgroup step loads a table of 64
      const int ntypes = c->labelled ? std::max(c->ll[l].ntypes, 64) : 64;
      lv.kinv = cv.take<char>((size_t)ntypes * 64 * es);
      std::vector<int> cells[27];
      const int nc = vanka_classes(p);
      Geom gh = lv.g;
      if (c->labelled) gh.flags = c->ll[l].flags.data();
      vanka_cells(gh, cells, nc == 27 ? 3 : 2);
      // the one-workgroup step keeps 64 types in LDS; the two-copy passes
      // resynchronise a band along the box walls only
      lv.sweep_ok = !c->labelled || c->ll[l].ntypes <= 64;
      long sum = 0;
      for (int k = 0; k < nc; ++k) {
        lv.nv[k] = (int)cells[k].size();
        if (nc == 8 && k >= 4)  // classes k and 7-k back to back: their pair pass reads one list
          lv.vcells[k] = lv.vcells[7 - k] ? lv.vcells[7 - k] + lv.nv[7 - k] : nullptr;
        else
          lv.vcells[k] =
              cv.take<int>(std::max<size_t>(cells[k].size() + (nc == 8 ? cells[7 - k].size() : 0), 1));
        lv.doff[k] = p.vanka == STOKES_VANKA_ADDITIVE ? sum : 0;
        sum += 8L * lv.nv[k];
        vmax = std::max<long>(vmax, p.vanka == STOKES_VANKA_ADDITIVE ? sum / 8 : lv.nv[k]);
      }
      if (nc == 8 && p.vanka != STOKES_VANKA_ADDITIVE)
        for (int q = 0; q < 4; ++q) vmax = std::max<long>(vmax, (long)lv.nv[q] + lv.nv[7 - q]);
      // two-copy passes where a pass is a latency chain (eight lanes per subdomain);
      // on larger levels the passes are bound by bandwidth and the copies cost more
      lv.pp = p.vanka == STOKES_VANKA_MULT8 && !c->labelled && !vsweep_level(lv, nc);
      for (int k = 0; k < nc; ++k) lv.pp = lv.pp && lv.nv[k] <= VANKA_LANES_MAX;
      if (lv.pp) lv.alt = cv.take<char>(tot * es);
      // the one-thread passes of a large box level run with the x-slabs set apart
      bool big = false;
      for (int k = 0; k < nc; ++k) big = big || lv.nv[k] > VANKA_LANES_MAX;
      if (big && p.vanka == STOKES_VANKA_MULT8 && !c->labelled && lv.g.nx >= 8)
        lv.xs = cv.take<char>(xslab_elems(lv.g) * es);
    }
  }
  c->vdelta = cv.take<char>(8 * std::max<long>(vmax, 1) * es);
  const Geom& gc = c->lev[L - 1].g;
  c->nc = c->labelled ? (int)c->ll[L - 1].n_dofs : (int)coarse_dofs(gc);
  c->cinv = cv.take<double>((size_t)c->nc * c->nc);
  c->cdof = cv.take<int>(c->nc);
}

// ---------------------------------------------------------------------------
// V-cycle pieces
// ---------------------------------------------------------------------------

// Every V-cycle launch goes through launch(): it runs `f` (which enqueues one
// kernel on c->ks), timing it with events when its class/level is selected.
// While a graph is being captured, a selected launch closes the running graph
// segment and is stored to run eagerly (between two segment replays) so its
// events sit on the caller's stream, outside any graph.
void seg_open(stokes_ctx* c);
void seg_close(stokes_ctx* c);

template <class F>
void launch(stokes_ctx* c, int cls, int level, F f) {
  if (c->prof_on(cls, level)) {
    if (c->capturing) {
      seg_close(c);
      stokes_ctx::Step st;
      st.fn = f;
      st.k = cls;
      st.l = level;
      c->steps.push_back(std::move(st));
      seg_open(c);
      return;
    }
    Prof pf(c, cls, level);
    f();
    return;
  }
  f();
}

// The cells of pair q (8 classes: classes q and 7-q, one list) and the class
// mask of its pass.
struct VPass {
  const int* cells;
  int n;
  int mask;
};
VPass vanka_pair_list(const Level& lv, int q) {
  return VPass{lv.vcells[q], lv.nv[q] + lv.nv[7 - q], vanka_pair8_mask(q)};
}

// Residual pass over n cells; corrections to vd (delta[r * n + c]).
template <typename T>
void vanka_delta_list(stokes_ctx* c, int l, const T* x, const T* b, const int* cells, int n, T* vd) {
  const Level& lv = c->lev[l];
  if (n == 0) return;
  const Geom g = lv.g;
  const T* kinv = (const T*)lv.kinv;
  if (n > VANKA_LANES_MAX) {  // one thread per subdomain
    const int nb = (n + BS - 1) / BS;
    launch(c, STOKES_KC_VANKA_DELTA, l,
           [=] { k_vanka_delta1<T, T><<<nb, BS, 0, c->ks>>>(g, x, b, cells, n, kinv, vd); });
  } else {  // eight lanes per subdomain
    const int nb = (8 * n + BS - 1) / BS;
    launch(c, STOKES_KC_VANKA_DELTA, l,
           [=] { k_vanka_delta<T, T><<<nb, BS, 0, c->ks>>>(g, x, b, cells, n, kinv, vd); });
  }
}

template <typename T>
void vanka_delta(stokes_ctx* c, int l, const T* x, const T* b, int k) {
  const Level& lv = c->lev[l];
  vanka_delta_list<T>(c, l, x, b, lv.vcells[k], lv.nv[k], (T*)c->vdelta + lv.doff[k]);
}

template <typename T>
void vanka_correct_list(stokes_ctx* c, int l, T* x, const int* cells, int n, const T* vd) {
  if (n == 0) return;
  const int nb = (8 * n + BS - 1) / BS;
  const Geom g = c->lev[l].g;
  launch(c, STOKES_KC_VANKA_APPLY, l, [=] { k_vanka_apply<T><<<nb, BS, 0, c->ks>>>(g, x, cells, n, vd); });
}

template <typename T>
void vanka_correct(stokes_ctx* c, int l, T* x, int k) {
  const Level& lv = c->lev[l];
  vanka_correct_list<T>(c, l, x, lv.vcells[k], lv.nv[k], (const T*)c->vdelta + lv.doff[k]);
}

// One application of the V1 smoother in a Vanka slot of Alg. 3: symmetric
// multiplicative Vanka (classes forward then backward, 8 classes as the
// complementary pairs of vanka_pair8; each pass from the state at its start),
// or additive Vanka (Eq. av: every class from the same
// state, the corrections then added class by class in a fixed order).
template <typename T>
void vanka_symmetric(stokes_ctx* c, int l, T* x, const T* b, XSlabCopy xin = XS_IN, bool xout = true) {
  const int nc = vanka_classes(c->prm);
  const Level& lv = c->lev[l];
  if (vsweep_level(lv, nc)) {  // small level: the whole step in one workgroup
    VSweep a{};
    a.g = lv.g;
    a.nc = nc;
    a.additive = c->prm.vanka == STOKES_VANKA_ADDITIVE;
    for (int k = 0; k < nc; ++k) {
      a.vc[k] = lv.vcells[k];
      a.nv[k] = lv.nv[k];
      a.doff[k] = lv.doff[k];
    }
    a.kinv = lv.kinv;
    if (!a.additive && 4L * lv.g.field <= vsweep_lds_elems<T>()) {  // the state fits in LDS
      launch(c, STOKES_KC_VANKA_DELTA, l, [=] { k_vanka_sweep_lds<T><<<1, VSWEEP_BS, 0, c->ks>>>(a, x, b); });
      return;
    }
    T* vd = (T*)c->vdelta;
    launch(c, STOKES_KC_VANKA_DELTA, l, [=] { k_vanka_sweep<T><<<1, VSWEEP_BS, 0, c->ks>>>(a, x, b, vd); });
    return;
  }
  if (c->prm.vanka == STOKES_VANKA_ADDITIVE) {
    for (int k = 0; k < nc; ++k) vanka_delta<T>(c, l, x, b, k);
    for (int k = 0; k < nc; ++k) vanka_correct<T>(c, l, x, k);
    return;
  }
  if (lv.pp) {  // two copies of the state; the 8 passes end in x
    const Geom g = lv.g;
    T* X[2] = {x, (T*)lv.alt};
    T* alt = X[1];
    // the second copy is brought up to date on the boundary band by the first
    // pass's launch; a level with a side below 8 copies its whole state first
    const bool band = std::min(g.nx, std::min(g.ny, g.nz)) >= 8;
    if (!band) {
      const long n = 4L * g.field;
      launch(c, STOKES_KC_VANKA_APPLY, l, [=] { k_convert<T, T><<<RED_BLOCKS, BS, 0, c->ks>>>(x, alt, n); });
    }
    const T* kinv = (const T*)lv.kinv;
    for (int pass = 0; pass < VANKA_PASSES8; ++pass) {
      const VPass cur = vanka_pair_list(lv, vanka_pair8(pass));
      // the previous pass's corrections to copy (none for the first pass and
      // for the second {3,4} pass)
      const int qp = vanka_pair8_prev(pass);
      const VPass prv = qp < 0 ? VPass{cur.cells, 0, 0} : vanka_pair_list(lv, qp);
      const int n = cur.n, np = prv.n, kmask = cur.mask;
      const int* cells = cur.cells;
      const int* prev = prv.cells;
      const T* R = X[pass & 1];
      T* W = X[(pass + 1) & 1];
      const int nband = band && pass == 0 ? (int)vanka_band_slots(g) : 0;
      if (n == 0 && np == 0 && nband == 0) continue;
      const int copy0 = (8 * n + 63) / 64 * 64;
      const int nb = (copy0 + 8 * np + nband + BS - 1) / BS;
      launch(c, STOKES_KC_VANKA_DELTA, l, [=] {
        k_vanka_pp8<T, T><<<nb, BS, 0, c->ks>>>(g, R, W, b, cells, n, kinv, prev, np, kmask, copy0, nband);
      });
    }
    return;
  }
  if (lv.xs) {  // classes forward then backward on the x-slabbed state
    const Geom g = lv.g;
    T* xs = (T*)lv.xs;
    const T* kinv = (const T*)lv.kinv;
    const int nbc = (int)((xslab_elems(g) + BS - 1) / BS);
    if (xin != XS_OUT)  // XS_OUT as the way in: the slab is current
      launch(c, STOKES_KC_VANKA_APPLY, l, [=] { k_xslab_copy<T><<<nbc, BS, 0, c->ks>>>(g, x, xs, xin); });
    for (int pass = 0; pass < VANKA_PASSES8; ++pass) {
      const VPass cur = vanka_pair_list(lv, vanka_pair8(pass));
      const int n = cur.n;
      if (n == 0) continue;
      const int* cells = cur.cells;
      T* vd = (T*)c->vdelta;
      launch(c, STOKES_KC_VANKA_DELTA, l, [=] {
        k_vanka_delta8_xs<T, T><<<(8 * n + BS - 1) / BS, BS, 0, c->ks>>>(g, x, xs, b, cells, n, kinv, vd);
      });
      launch(c, STOKES_KC_VANKA_APPLY, l,
             [=] { k_vanka_apply_xs<T><<<(8 * n + BS - 1) / BS, BS, 0, c->ks>>>(g, x, xs, cells, n, vd); });
    }
    if (xout) launch(c, STOKES_KC_VANKA_APPLY, l, [=] { k_xslab_copy<T><<<nbc, BS, 0, c->ks>>>(g, x, xs, XS_OUT); });
    return;
  }
  if (nc == 8) {
    for (int pass = 0; pass < VANKA_PASSES8; ++pass) {
      const VPass cur = vanka_pair_list(lv, vanka_pair8(pass));
      vanka_delta_list<T>(c, l, x, b, cur.cells, cur.n, (T*)c->vdelta);
      vanka_correct_list<T>(c, l, x, cur.cells, cur.n, (const T*)c->vdelta);
    }
    return;
  }
  for (int pass = 0; pass < 2 * nc; ++pass) {
    const int k = pass < nc ? pass : 2 * nc - 1 - pass;
    vanka_delta<T>(c, l, x, b, k);
    vanka_correct<T>(c, l, x, k);
  }
}

// Forward DGS sweep on L~ M (Alg. 2, Eq. dist) over the V2 unknowns:
// velocities red, black; then the pressures by the eight colour classes 0..7,
// run as four stages of equal bit count (packed_kernels.hpp) in five launches:
// launch t makes the stage-t own steps and the stage-(t-1) neighbour updates.
template <typename T>
void dgs_forward(stokes_ctx* c, int l, T* x, const T* b) {
  constexpr int V = dgs_pack<T>();
  const Geom g = c->lev[l].g;
  T* dscr = (T*)c->lev[l].dscr;
  if (dgs_small_packs<V>(g) <= DSWEEP_MAX_PACKS) {  // small level: the sweep in one workgroup
    launch(c, STOKES_KC_DGS_U, l, [=] { k_dgs_small<T, T, V><<<1, DSWEEP_BS, 0, c->ks>>>(g, x, b, dscr, 0); });
    return;
  }
  const int hg = dgs_grid<T>(g);
  for (int col = 0; col < 2; ++col)
    launch(c, STOKES_KC_DGS_U, l, [=] { k_dgs_u_v<T, T, V><<<hg, BS, 0, c->ks>>>(g, x, b, col); });
  for (int t = 0; t <= 4; ++t)
    launch(c, t < 4 ? STOKES_KC_DGS_PF_OWN : STOKES_KC_DGS_PF_NBR, l,
           [=] { k_dgs_pf_v<T, T, V><<<hg, BS, 0, c->ks>>>(g, x, b, dscr, t); });
}

// Reverse sweep: Gauss-Seidel on M^T L~ (Eq. ldist) in exactly the reverse
// order: pressure stages 3, 2, 1, 0 (classes 7..0); velocities black, red.
template <typename T>
void dgs_reverse(stokes_ctx* c, int l, T* x, const T* b) {
  constexpr int V = dgs_pack<T>();
  const Geom g = c->lev[l].g;
  if (dgs_small_packs<V>(g) <= DSWEEP_MAX_PACKS) {  // small level: the sweep in one workgroup
    T* dscr = (T*)c->lev[l].dscr;
    launch(c, STOKES_KC_DGS_U, l, [=] { k_dgs_small<T, T, V><<<1, DSWEEP_BS, 0, c->ks>>>(g, x, b, dscr, 1); });
    return;
  }
  const int hg = dgs_grid<T>(g);
  for (int st = 3; st >= 0; --st)
    launch(c, STOKES_KC_DGS_PR, l, [=] { k_dgs_pr_v<T, T, V><<<hg, BS, 0, c->ks>>>(g, x, b, st); });
  for (int col = 1; col >= 0; --col)
    launch(c, STOKES_KC_DGS_U, l, [=] { k_dgs_u_v<T, T, V><<<hg, BS, 0, c->ks>>>(g, x, b, col); });
}

enum Interior { INT_SYMMETRIC, INT_REVERSE, INT_FORWARD };

// Alg. 3: symmetric Vanka on V1, interior smoother on V2, symmetric Vanka on V1.
// On a level with an x-slab, `first` says what the slab needs before the
// first Vanka step: XS_ZERO (x is 0), XS_IN (x changed) or XS_OUT (nothing
// changed since the last step wrote the slab back).  Consecutive Vanka steps
// share the slab; the DGS sweeps between change it (the pressure steps of V2
// cells move the faces and pressures beside them).
template <typename T>
void smooth(stokes_ctx* c, int l, T* x, const T* b, Interior kind, int sweeps, XSlabCopy first) {
  const int nb = c->prm.n_boundary;
  for (int i = 0; i < nb; ++i) vanka_symmetric(c, l, x, b, i == 0 ? first : XS_OUT, i == nb - 1);
  for (int i = 0; i < sweeps; ++i) {
    if (kind != INT_FORWARD) {
      if (kind == INT_SYMMETRIC) dgs_forward(c, l, x, b);
      dgs_reverse(c, l, x, b);
    } else {
      dgs_forward(c, l, x, b);
    }
  }
  for (int i = 0; i < nb; ++i)
    vanka_symmetric(c, l, x, b, i == 0 && sweeps > 0 ? XS_IN : XS_OUT, i == nb - 1);
}

template <typename T>
void presmooth(stokes_ctx* c, int l, T* x, const T* b, bool x_zero) {
  const XSlabCopy first = x_zero ? XS_ZERO : XS_IN;
  if (c->prm.smoother == STOKES_SMOOTHER_SYMMETRIC) {
    for (int i = 0; i < c->prm.nu / 2; ++i) smooth(c, l, x, b, INT_SYMMETRIC, 1, i == 0 ? first : XS_OUT);
  } else {
    smooth(c, l, x, b, INT_REVERSE, c->prm.nu, first);
  }
}

template <typename T>
void postsmooth(stokes_ctx* c, int l, T* x, const T* b) {
  if (c->prm.smoother == STOKES_SMOOTHER_SYMMETRIC) {
    for (int i = 0; i < c->prm.nu / 2; ++i) smooth(c, l, x, b, INT_SYMMETRIC, 1, i == 0 ? XS_IN : XS_OUT);
  } else {
    smooth(c, l, x, b, INT_FORWARD, c->prm.nu, XS_IN);
  }
}

template <typename T>
void fill_zero(stokes_ctx* c, T* x, long n, int level = 0) {
  launch(c, STOKES_KC_BLAS, level, [=] { k_fill<T><<<RED_BLOCKS, BS, 0, c->ks>>>(x, n, T(0)); });
}

// x = V-CYCLE(L~, b, 0, L - l) (from the current x when zero_init is false);
// with cycle = 2 the coarse correction is two cycles (a W-cycle)
template <typename T>
void vcycle(stokes_ctx* c, int l, const T* b, T* x, bool zero_init = true) {
  const Geom g = c->lev[l].g;
  if (zero_init) fill_zero(c, x, 4L * g.field, l);
  if (l == c->L - 1) {
    const int nb = (c->nc + (BS / 64) - 1) / (BS / 64);
    const double* cinv = c->cinv;
    const int* cdof = c->cdof;
    const int nc = c->nc;
    launch(c, STOKES_KC_COARSE, l, [=] { k_coarse_solve<T><<<nb, BS, 0, c->ks>>>(cinv, cdof, nc, b, x); });
    return;
  }
  presmooth(c, l, x, b, zero_init);
  const Geom gc = c->lev[l + 1].g;
  T* bc = (T*)c->lev[l + 1].b;
  T* xc = (T*)c->lev[l + 1].x;
  {  // coarse b = R (b - L~ x) without the fine residual in memory
    T* S = (T*)c->lev[l].r;
    const int gxy = (int)rr_blocks(g, gc);
    launch(c, STOKES_KC_RESTRICT, l, [=] {
      k_resid_restrict_xy<T, dgs_pack<T>()><<<gxy, BS, 0, c->ks>>>(g, gc, x, b, S);
    });
    launch(c, STOKES_KC_RESTRICT, l, [=] { k_restrict_z<T><<<restrict_grid(gc), BS, 0, c->ks>>>(g, gc, S, bc); });
  }
  vcycle(c, l + 1, (const T*)bc, xc);
  for (int i = 1; i < c->prm.cycle; ++i) vcycle(c, l + 1, (const T*)bc, xc, false);
  launch(c, STOKES_KC_PROLONG, l, [=] { k_prolong_pairs<T><<<prolong_grid(gc), BS, 0, c->ks>>>(g, gc, xc, x); });
  if (c->labelled)
    launch(c, STOKES_KC_PROLONG, l, [=] { k_prolong_edge<T><<<prolong_edge_grid(g), BS, 0, c->ks>>>(g, gc, xc, x); });
  postsmooth(c, l, x, b);
}

// FP32 V-cycle: its right-hand side is already in the float level buffer
// (written with s), and/or its result is left there for the SQMR passes,
// which read it as float, instead of converting it into t.
enum { PC_IN_READY = 1, PC_OUT_FLOAT = 2 };

// The whole preconditioner application t = W s: FP64 runs the V-cycle on the
// caller's vectors; FP32 converts s once, runs the V-cycle on float level
// buffers (all smoother, transfer and stencil arithmetic in FP32; the
// coarsest solve accumulates in FP64) and converts the result back (io: the
// PC_* flags).
void precondition(stokes_ctx* c, const double* s, double* t, int io = 0) {
  if (c->prec == 64) {
    vcycle<double>(c, 0, s, t);
    return;
  }
  float* b0 = (float*)c->lev[0].b;
  float* x0 = (float*)c->lev[0].x;
  const long n = c->total;
  if (!(io & PC_IN_READY))
    launch(c, STOKES_KC_BLAS, 0, [=] { k_convert<double, float><<<RED_BLOCKS, BS, 0, c->ks>>>(s, b0, n); });
  vcycle<float>(c, 0, b0, x0);
  if (!(io & PC_OUT_FLOAT))
    launch(c, STOKES_KC_BLAS, 0, [=] { k_convert<float, double><<<RED_BLOCKS, BS, 0, c->ks>>>(x0, t, n); });
}

void seg_open(stokes_ctx* c) {
  if (c->cap_error == hipSuccess) c->cap_error = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
}

void seg_close(stokes_ctx* c) {
  if (c->cap_error != hipSuccess) return;
  hipGraph_t graph = nullptr;
  c->cap_error = hipStreamEndCapture(c->cap, &graph);
  if (c->cap_error != hipSuccess) return;
  size_t nodes = 0;
  (void)hipGraphGetNodes(graph, nullptr, &nodes);
  if (nodes == 0) {
    (void)hipGraphDestroy(graph);
    return;
  }
  stokes_ctx::Step st;
  st.graph = graph;
  c->cap_error = hipGraphInstantiate(&st.exec, graph, nullptr, nullptr, 0);
  c->steps.push_back(std::move(st));
}

// t = W s on the caller's stream.  The V-cycle (about 900 launches at 256^3)
// is captured once per (s, t, profiling selection) into graph segments that
// are replayed on the caller's stream; STOKES_FLAG_NO_GRAPH launches it
// kernel by kernel instead.
int run_vcycle(stokes_ctx* c, const double* s, double* t, int io = 0) {
  if (c->prec == 64) io = 0;
  if (c->prm.flags & STOKES_FLAG_NO_GRAPH) {
    c->ks = c->stream;
    precondition(c, s, t, io);
    return hipGetLastError() == hipSuccess ? STOKES_OK : STOKES_EDEVICE;
  }
  stokes_ctx::GraphEntry* hit = nullptr;
  for (auto& e : c->graphs)
    if (e.s == s && e.t == t && e.pc == c->prof_class && e.pl == c->prof_level && e.io == io) hit = &e;
  if (!hit) {
    if (c->graphs.size() >= 4) {
      (void)hipStreamSynchronize(c->stream);
      drop_graphs(c);
    }
    c->steps.clear();
    c->cap_error = hipSuccess;
    c->capturing = true;
    c->ks = c->cap;
    seg_open(c);
    precondition(c, s, t, io);
    seg_close(c);
    c->capturing = false;
    c->ks = c->stream;
    stokes_ctx::GraphEntry e{s, t, c->prof_class, c->prof_level, io, std::move(c->steps)};
    c->steps.clear();
    c->graphs.push_back(std::move(e));
    hit = &c->graphs.back();
    if (c->cap_error != hipSuccess || hipGetLastError() != hipSuccess) {
      drop_graphs(c);
      return STOKES_EDEVICE;
    }
  }
  for (auto& st : hit->steps) {
    if (st.exec) {
      if (hipGraphLaunch(st.exec, c->stream) != hipSuccess) return STOKES_EDEVICE;
    } else {
      Prof pf(c, st.k, st.l);
      st.fn();
    }
  }
  return hipGetLastError() == hipSuccess ? STOKES_OK : STOKES_EDEVICE;
}

// Device scalar reduction of `nblk` partials (stride values each) into
// dscal[0..stride), copied to the pinned host mirror and waited for.
int reduce_to_host(stokes_ctx* c, int nblk, int stride) {
  {
    Prof pf(c, STOKES_KC_BLAS, 0);
    k_reduce<<<1, 1024, 0, c->stream>>>(c->partial, nblk, stride, c->dscal);
  }
  HIPCHK(hipMemcpyAsync(c->hscal, c->dscal, sizeof(double) * stride, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (!c->pending.empty()) prof_collect(c);
  return STOKES_OK;
}

}  // namespace

namespace {

// Set-up of a context on `workspace`.  With on_static the workspace is the
// library's static scratch and the context allocates nothing: no pinned host
// mirror (the scalars come back into the context itself), no capture stream,
// no graphs (its V-cycles launch kernel by kernel).
int setup_ctx(const stokes_params* p, void* workspace, size_t bytes, void* hip_stream, bool on_static,
              stokes_ctx** out) {
  if (!out) return STOKES_EINVAL;
  *out = nullptr;
  int L = 0;
  int st = validate(p, &L);
  if (st != STOKES_OK) return st;
  size_t need = 0;
  stokes_workspace_bytes(p, &need);
  if (!workspace || bytes < need || ((uintptr_t)workspace & 255)) return STOKES_EINVAL;
  stokes_ctx* c = new (std::nothrow) stokes_ctx();
  if (!c) return STOKES_EINVAL;
  c->prm = *p;
  c->L = L;
  c->stream = (hipStream_t)hip_stream;
  c->ks = c->stream;
  c->on_static = on_static;
  Carver cv(workspace, bytes, false);
  carve(c, cv, L);
  if (on_static) {
    c->prm.flags |= STOKES_FLAG_NO_GRAPH;
    c->hscal = c->hscal_local;
  } else {
    if (hipHostMalloc((void**)&c->hscal, sizeof(double) * 16, hipHostMallocDefault) != hipSuccess) {
      delete c;
      return STOKES_EDEVICE;
    }
    if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
      (void)hipHostFree(c->hscal);
      delete c;
      return STOKES_EDEVICE;
    }
  }
  // Host tables, uploaded with synchronous waits so the host buffers can go.
  auto fail = [&](int code) {
    stokes_destroy(c);
    return code;
  };
  if (c->labelled) {
    for (int l = 0; l < L; ++l) {
      Level& lv = c->lev[l];
      if (c->ll[l].ntypes > 1024 ||
          hipMemcpyAsync(lv.flags, c->ll[l].flags.data(), sizeof(uint32_t) * lv.g.field, hipMemcpyHostToDevice,
                         c->stream) != hipSuccess)
        return fail(STOKES_EDEVICE);
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(STOKES_EDEVICE);
  }
  for (int l = 0; l < L - 1; ++l) {
    Level& lv = c->lev[l];
    std::vector<double> kinv;
    if (c->labelled) {
      kinv = c->ll[l].kinv;
      if (kinv.empty()) kinv.assign(64, 0.0);
    } else if (!vanka_inverses(lv.g, kinv)) {
      return fail(STOKES_EINVAL);
    }
    std::vector<float> kinv_f(kinv.begin(), kinv.end());
    const void* src = c->prec == 32 ? (const void*)kinv_f.data() : (const void*)kinv.data();
    const size_t nbytes = kinv.size() * (c->prec == 32 ? sizeof(float) : sizeof(double));
    if (hipMemcpyAsync(lv.kinv, src, nbytes, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return fail(STOKES_EDEVICE);
    std::vector<int> cells[27];
    const int nc = vanka_classes(c->prm);
    Geom gh = lv.g;
    if (c->labelled) gh.flags = c->ll[l].flags.data();
    vanka_cells(gh, cells, nc == 27 ? 3 : 2);
    for (int k = 0; k < nc; ++k) {
      if (cells[k].empty()) continue;
      if (hipMemcpyAsync(lv.vcells[k], cells[k].data(), cells[k].size() * sizeof(int), hipMemcpyHostToDevice,
                         c->stream) != hipSuccess)
        return fail(STOKES_EDEVICE);
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(STOKES_EDEVICE);
  }
  {
    std::vector<int> dof;
    std::vector<double> inv;
    Geom gh = c->lev[L - 1].g;
    if (c->labelled) gh.flags = c->ll[L - 1].flags.data();
    if (!coarse_inverse(gh, dof, inv) || (int)dof.size() != c->nc) return fail(STOKES_EINVAL);
    if (hipMemcpyAsync(c->cinv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice, c->stream) !=
            hipSuccess ||
        hipMemcpyAsync(c->cdof, dof.data(), dof.size() * sizeof(int), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return fail(STOKES_EDEVICE);
  }
  // kernels of a labelled domain read its flag words
  if (c->labelled)
    for (int l = 0; l < L; ++l) c->lev[l].g.flags = c->lev[l].flags;
  c->labs.clear();
  c->labs.shrink_to_fit();
  for (auto& t : c->ll) {
    t.flags.clear();
    t.flags.shrink_to_fit();
    t.kinv.clear();
  }
  // workspace vectors start from zero (their ghost slots are never written otherwise)
  for (int l = 0; l < L; ++l) {
    if (!c->lev[l].b) continue;
    const long n = 4L * c->lev[l].g.field;
    if (c->prec == 32) {
      fill_zero(c, (float*)c->lev[l].b, n);
      fill_zero(c, (float*)c->lev[l].x, n);
    } else {
      fill_zero(c, (double*)c->lev[l].b, n);
      fill_zero(c, (double*)c->lev[l].x, n);
    }
  }
  fill_zero(c, c->s, c->total);
  fill_zero(c, c->t, c->total);
  fill_zero(c, c->q, c->total);
  fill_zero(c, c->d, c->total);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) return fail(STOKES_EDEVICE);
  *out = c;
  return STOKES_OK;
}

}  // namespace

// The static scratch of stokes_solve_static: a file-scope device array, one
// copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel or a copy (in host code it is only a stand-in for
// the symbol): it looks the device address up once per device, with that
// device current, and uses that pointer.
static __device__ __align__(256) unsigned char scratch[STOKES_STATIC_BYTES];

namespace {

constexpr int STATIC_MAX_DEVICES = 64;
std::mutex g_static_mu;
void* g_static_ptr[STATIC_MAX_DEVICES] = {};

int static_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= STATIC_MAX_DEVICES) return STOKES_EDEVICE;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return STOKES_EDEVICE;
    g_static_ptr[dev] = ptr;
  }
  *out = g_static_ptr[dev];
  return STOKES_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int stokes_default_params(int32_t nx, int32_t ny, int32_t nz, double h, stokes_params* p) {
  if (!p) return STOKES_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->nx = nx;
  p->ny = ny;
  p->nz = nz;
  p->h = h;
  p->eta = 1.0;
  p->gamma = 1e-3;
  p->levels = 0;
  p->nu = 2;
  p->n_boundary = 1;
  p->vcycle_precision = 64;
  p->smoother = STOKES_SMOOTHER_SYMMETRIC;
  p->flags = STOKES_FLAG_REMOVE_MEAN;
  p->vanka = STOKES_VANKA_MULT8;
  p->cycle = 1;
  return STOKES_OK;
}

int stokes_workspace_bytes(const stokes_params* p, size_t* bytes) {
  int L = 0;
  const int st = validate(p, &L);
  if (st != STOKES_OK) return st;
  if (!bytes) return STOKES_EINVAL;
  stokes_ctx tmp;
  tmp.prm = *p;
  Carver cv(nullptr, 0, true);
  carve(&tmp, cv, L);
  *bytes = (cv.used + 255) & ~size_t(255);
  return STOKES_OK;
}

int stokes_setup(const stokes_params* p, void* workspace, size_t bytes, void* hip_stream, stokes_ctx** out) {
  return setup_ctx(p, workspace, bytes, hip_stream, false, out);
}


int stokes_layout(const stokes_ctx* c, stokes_layout_t* out) {
  if (!c || !out) return STOKES_EINVAL;
  const Geom& g = c->lev[0].g;
  out->nx = g.nx;
  out->ny = g.ny;
  out->nz = g.nz;
  out->sy = g.sy;
  out->sz = g.sz;
  for (int f = 0; f < 4; ++f) out->off[f] = (int64_t)f * g.field;
  out->field = g.field;
  out->total = c->total;
  out->n_dofs = c->labelled ? c->ll[0].n_dofs : coarse_dofs(g);
  out->levels = c->L;
  return STOKES_OK;
}

int stokes_level_layout(const stokes_ctx* c, int32_t level, stokes_layout_t* out) {
  if (!c || !out || level < 0 || level >= c->L) return STOKES_EINVAL;
  const Geom& g = c->lev[level].g;
  out->nx = g.nx;
  out->ny = g.ny;
  out->nz = g.nz;
  out->sy = g.sy;
  out->sz = g.sz;
  for (int f = 0; f < 4; ++f) out->off[f] = (int64_t)f * g.field;
  out->field = g.field;
  out->total = 4L * g.field;
  out->n_dofs = c->labelled ? c->ll[level].n_dofs : coarse_dofs(g);
  out->levels = c->L - level;
  return STOKES_OK;
}

int stokes_restrict(stokes_ctx* c, const double* fine, double* coarse) {
  if (!c || !fine || !coarse || fine == coarse || c->L < 2) return STOKES_EINVAL;
  const Geom& g = c->lev[0].g;
  const Geom& gc = c->lev[1].g;
  k_restrict<double><<<restrict_grid(gc), BS, 0, c->stream>>>(g, gc, fine, coarse);
  return hipGetLastError() == hipSuccess ? STOKES_OK : STOKES_EDEVICE;
}

int stokes_prolong(stokes_ctx* c, const double* coarse, double* fine) {
  if (!c || !fine || !coarse || fine == coarse || c->L < 2) return STOKES_EINVAL;
  const Geom& g = c->lev[0].g;
  const Geom& gc = c->lev[1].g;
  k_fill<double><<<RED_BLOCKS, BS, 0, c->stream>>>(fine, 4L * g.field, 0.0);
  k_prolong_pairs<double><<<prolong_grid(gc), BS, 0, c->stream>>>(g, gc, coarse, fine);
  if (c->labelled) k_prolong_edge<double><<<prolong_edge_grid(g), BS, 0, c->stream>>>(g, gc, coarse, fine);
  return hipGetLastError() == hipSuccess ? STOKES_OK : STOKES_EDEVICE;
}

int stokes_lift(stokes_ctx* c, const double* g, const double* b, double* out) {
  if (!c || !g || !b || !out || g == out || b == out) return STOKES_EINVAL;
  const Geom& ge = c->lev[0].g;
  // b - L g at the unknowns (g holds the boundary values outside them), 0 elsewhere
  k_apply_v<AP_RESID, double, double, 2><<<apply_grid<double>(ge), BS, 0, c->stream>>>(ge, g, b, out, 0.0, nullptr);
  return hipGetLastError() == hipSuccess ? STOKES_OK : STOKES_EDEVICE;
}

int stokes_apply(stokes_ctx* c, const double* x, double* y, int32_t penalized) {
  if (!c || !x || !y || x == y) return STOKES_EINVAL;
  const Geom& g = c->lev[0].g;
  {
    Prof pf(c, STOKES_KC_APPLY, 0);
    k_apply_v<AP_APPLY, double, double, 2><<<apply_grid<double>(g), BS, 0, c->stream>>>(g, x, (const double*)nullptr, y,
                                                                               penalized ? g.gamma : 0.0, nullptr);
  }
  return hipGetLastError() == hipSuccess ? STOKES_OK : STOKES_EDEVICE;
}

int stokes_vcycle(stokes_ctx* c, const double* s, double* t) {
  if (!c || !s || !t || s == t) return STOKES_EINVAL;
  return run_vcycle(c, s, t);
}

int stokes_solve(stokes_ctx* c, const double* b, double* x, double rtol, int32_t maxit, stokes_info* info) {
  if (!c || !b || !x || b == x || maxit < 0 || !(rtol >= 0)) return STOKES_EINVAL;
  const Geom& g = c->lev[0].g;
  const long n = c->total;
  const int gf = grid_for(g.field);  // flat kernels (ghost clearing, pressure mean)
  const int ga = apply_grid<double>(g);  // packed operator kernels
  auto fill_info = [&](int iters, int status, double relres, double bn) {
    if (info) {
      info->iters = iters;
      info->status = status;
      info->relres = relres;
      info->bnorm = bn;
    }
    return status;
  };
  {
    Prof pf(c, STOKES_KC_BLAS, 0);
    k_clear_ghosts<<<gf, BS, 0, c->stream>>>(g, x);
  }
  // ||b|| over the unknowns
  {
    Prof pf(c, STOKES_KC_APPLY, 0);
    k_apply_v<AP_BNORM, double, double, 2><<<ga, BS, 0, c->stream>>>(g, (const double*)nullptr, b, (double*)nullptr, 0.0,
                                                                c->partial);
  }
  if (reduce_to_host(c, ga, 1) != STOKES_OK) return fill_info(0, STOKES_EDEVICE, NAN, NAN);
  const double bnorm = std::sqrt(c->hscal[0]);
  if (!std::isfinite(bnorm)) return fill_info(0, STOKES_ENONFINITE, NAN, bnorm);
  if (bnorm == 0.0) {
    fill_zero(c, x, n);
    if (info && info->history) info->history[0] = 0.0;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fill_info(0, STOKES_EDEVICE, 0.0, 0.0);
    return fill_info(0, STOKES_OK, 0.0, 0.0);
  }
  // s0 = b - L x0, with ||s0||^2
  {
    Prof pf(c, STOKES_KC_APPLY, 0);
    k_apply_v<AP_RESID, double, double, 2><<<ga, BS, 0, c->stream>>>(g, x, b, c->s, 0.0, nullptr);
  }
  {
    Prof pf(c, STOKES_KC_APPLY, 0);
    k_apply_v<AP_RESNORM, double, double, 2><<<ga, BS, 0, c->stream>>>(g, x, b, (double*)nullptr, 0.0, c->partial);
  }
  if (reduce_to_host(c, ga, 1) != STOKES_OK) return fill_info(0, STOKES_EDEVICE, NAN, bnorm);
  double relres = std::sqrt(c->hscal[0]) / bnorm;
  if (info && info->history) info->history[0] = relres;
  auto finish = [&](int iters, int status) {
    if (status == STOKES_OK && (c->prm.flags & STOKES_FLAG_REMOVE_MEAN) && !c->neumann) {
      {
        Prof pf(c, STOKES_KC_BLAS, 0);
        k_sum_p<<<gf, BS, 0, c->stream>>>(g, x, c->partial);
      }
      {
        Prof pf(c, STOKES_KC_BLAS, 0);
        k_reduce<<<1, 1024, 0, c->stream>>>(c->partial, gf, 1, c->dscal);
      }
      const double ncell = c->labelled ? (double)c->ll[0].n_cells : (double)g.nx * g.ny * g.nz;
      // mean = sum / ncell, computed on the host to keep one rounding
      if (hipMemcpyAsync(c->hscal, c->dscal, sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
          hipStreamSynchronize(c->stream) != hipSuccess)
        return fill_info(iters, STOKES_EDEVICE, relres, bnorm);
      const double mean = c->hscal[0] / ncell;
      {
        Prof pf(c, STOKES_KC_BLAS, 0);
        k_shift_p<<<gf, BS, 0, c->stream>>>(g, x, mean);
      }
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
      return fill_info(iters, STOKES_EDEVICE, relres, bnorm);
    return fill_info(iters, status, relres, bnorm);
  };
  if (!std::isfinite(relres)) return finish(0, STOKES_ENONFINITE);
  if (relres <= rtol) return finish(0, STOKES_OK);
  // t = W s0; q0 = t; tau0 = ||t||; rho0 = s0 . q0; d = 0
  if (run_vcycle(c, c->s, c->t) != STOKES_OK) return finish(0, STOKES_EDEVICE);
  {
    Prof pf(c, STOKES_KC_BLAS, 0);
    k_dot_aa_ac<double><<<RED_BLOCKS, BS, 0, c->stream>>>(c->t, c->s, n, c->partial);
  }
  if (reduce_to_host(c, RED_BLOCKS, 2) != STOKES_OK) return finish(0, STOKES_EDEVICE);
  double tau = std::sqrt(c->hscal[0]);
  double rho = c->hscal[1];
  HIPCHK(hipMemcpyAsync(c->q, c->t, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  fill_zero(c, c->d, n);
  double nu_prev = 0.0;
  for (int j = 1; j <= maxit; ++j) {
    // t = L q, sigma = q . t
    {
      Prof pf(c, STOKES_KC_APPLY, 0);
      k_apply_v<AP_APPLY_DOT, double, double, 2><<<ga, BS, 0, c->stream>>>(g, c->q, (const double*)nullptr, c->t, 0.0,
                                                                      c->partial);
    }
    if (reduce_to_host(c, ga, 1) != STOKES_OK) return finish(j - 1, STOKES_EDEVICE);
    const double sigma = c->hscal[0];
    if (!std::isfinite(sigma)) return finish(j - 1, STOKES_ENONFINITE);
    if (sigma == 0.0) return finish(j - 1, STOKES_EBREAKDOWN);
    const double alpha = rho / sigma;
    // FP32 V-cycle: the s update also writes its float right-hand side, and
    // W s stays in the float level buffer, where the next two passes read it
    float* const wf = c->prec == 32 ? (float*)c->lev[0].x : nullptr;
    {
      Prof pf(c, STOKES_KC_BLAS, 0);
      k_axpy_neg<<<RED_BLOCKS, BS, 0, c->stream>>>(c->s, c->t, n, alpha, wf ? (float*)c->lev[0].b : nullptr);
    }
    // t = W s
    if (run_vcycle(c, c->s, c->t, wf ? PC_IN_READY | PC_OUT_FLOAT : 0) != STOKES_OK)
      return finish(j - 1, STOKES_EDEVICE);
    {
      Prof pf(c, STOKES_KC_BLAS, 0);
      if (wf)
        k_dot_aa_ac<float><<<RED_BLOCKS, BS, 0, c->stream>>>(wf, c->s, n, c->partial);
      else
        k_dot_aa_ac<double><<<RED_BLOCKS, BS, 0, c->stream>>>(c->t, c->s, n, c->partial);
    }
    if (reduce_to_host(c, RED_BLOCKS, 2) != STOKES_OK) return finish(j - 1, STOKES_EDEVICE);
    const double tnorm = std::sqrt(c->hscal[0]);
    const double rho_new = c->hscal[1];
    const double nu = tnorm / tau;
    const double cc = 1.0 / std::sqrt(1.0 + nu * nu);
    tau = tau * nu * cc;
    {
      Prof pf(c, STOKES_KC_BLAS, 0);
      // with the next direction q = t + (rho_new / rho) q in the same pass (unused when the loop ends here)
      if (wf)
        k_update_dxq<float><<<RED_BLOCKS, BS, 0, c->stream>>>(c->d, c->q, x, wf, n, cc * cc * nu_prev * nu_prev,
                                                              cc * cc * alpha, rho_new / rho);
      else
        k_update_dxq<double><<<RED_BLOCKS, BS, 0, c->stream>>>(c->d, c->q, x, c->t, n, cc * cc * nu_prev * nu_prev,
                                                               cc * cc * alpha, rho_new / rho);
    }
    nu_prev = nu;
    // true residual
    {
      Prof pf(c, STOKES_KC_APPLY, 0);
      k_apply_v<AP_RESNORM, double, double, 2><<<ga, BS, 0, c->stream>>>(g, x, b, (double*)nullptr, 0.0, c->partial);
    }
    if (reduce_to_host(c, ga, 1) != STOKES_OK) return finish(j, STOKES_EDEVICE);
    relres = std::sqrt(c->hscal[0]) / bnorm;
    if (info && info->history) info->history[j] = relres;
    if (!std::isfinite(relres) || !std::isfinite(tnorm)) return finish(j, STOKES_ENONFINITE);
    if (relres <= rtol) return finish(j, STOKES_OK);
    if (rho == 0.0) return finish(j, STOKES_EBREAKDOWN);
    rho = rho_new;
  }
  return finish(maxit, STOKES_ENOCONV);
}

int stokes_profile(stokes_ctx* c, int32_t kernel_class, int32_t level) {
  if (!c || kernel_class < STOKES_KC_OFF || kernel_class >= STOKES_KC_COUNT || level >= 32) return STOKES_EINVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return STOKES_EDEVICE;
  prof_collect(c);
  if (kernel_class != c->prof_class || level != c->prof_level) drop_graphs(c);
  c->prof_class = kernel_class;
  c->prof_level = level;
  c->prof_ms.assign(STOKES_KC_COUNT * 32, 0.0);
  c->prof_n.assign(STOKES_KC_COUNT * 32, 0);
  return STOKES_OK;
}

int stokes_profile_read(stokes_ctx* c, int32_t kernel_class, int32_t level, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches || kernel_class < 0 || kernel_class >= STOKES_KC_COUNT || level >= 32)
    return STOKES_EINVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return STOKES_EDEVICE;
  prof_collect(c);
  double ms = 0.0;
  long n = 0;
  if (!c->prof_ms.empty()) {
    for (int l = 0; l < 32; ++l) {
      if (level >= 0 && l != level) continue;
      ms += c->prof_ms[kernel_class * 32 + l];
      n += c->prof_n[kernel_class * 32 + l];
    }
  }
  *total_ms = ms;
  *launches = n;
  return STOKES_OK;
}

void stokes_destroy(stokes_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  prof_collect(c);
  drop_graphs(c);
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->hscal && !c->on_static) (void)hipHostFree(c->hscal);
  delete c;
}

int stokes_solve_static(const stokes_params* p, const double* b, double* x, double rtol, int32_t maxit,
                        stokes_info* info, void* hip_stream) {
  int L = 0;
  const int st = validate(p, &L);
  if (st != STOKES_OK) return st;
  size_t need = 0;
  stokes_workspace_bytes(p, &need);
  if (need > STOKES_STATIC_BYTES) return STOKES_ETOOLARGE;
  if (!b || !x || b == x || maxit < 0 || !(rtol >= 0)) return STOKES_EINVAL;
  void* ws = nullptr;
  if (static_scratch(&ws) != STOKES_OK) return STOKES_EDEVICE;
  stokes_ctx* c = nullptr;
  const int rc = setup_ctx(p, ws, STOKES_STATIC_BYTES, hip_stream, true, &c);
  if (rc != STOKES_OK) return rc;
  const int status = stokes_solve(c, b, x, rtol, maxit, info);
  stokes_destroy(c);
  return status;
}

const char* stokes_strerror(int status) {
  switch (status) {
    case STOKES_OK: return "ok";
    case STOKES_EINVAL: return "invalid argument (dimensions, levels, pointer, alignment or workspace size)";
    case STOKES_ENOCONV: return "not converged within maxit iterations";
    case STOKES_EBREAKDOWN: return "SQMR breakdown (sigma or rho is zero)";
    case STOKES_ENONFINITE: return "non-finite value in the iteration";
    case STOKES_EDEVICE: return "HIP runtime error";
    case STOKES_ETOOLARGE: return "problem too large for the static scratch of stokes_solve_static";
    default: return "unknown status";
  }
}

}  // extern "C"
