// Batched MG-SQMR: many independent box domains solved together on one GPU.
//
// Every kernel launch covers one step of the method for all domains that take
// part in it (one table entry per domain, see batched_kernels.hpp), so the
// launch count of a batch equals that of a single solve of its deepest
// domain.  The SQMR recurrences of Alg. 4 run per domain on the device (one
// thread per domain for the scalars, segmented fixed-order reductions for the
// inner products); a domain that has converged, broken down or run out of
// iterations drops out of every later launch.  The set-up phase and each
// chunk of iterations are captured as HIP graphs on a private stream and
// replayed on the caller's stream; the host reads one counter per replay.
//
// Tile shapes: the stencil kernels take a 2-D tile of BX x (256/BX) items per
// block; stokes_batch_autotune() times every BX on every level of the batch
// and keeps the fastest per kernel class and level.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <thread>
#include <vector>

#include "batched_kernels.hpp"
#include "host_tables.hpp"
#include "stokes_mgsqmr.h"

using namespace sg;

namespace {

constexpr int NBX = 4;
constexpr int BXV[NBX] = {32, 64, 128, 256};
enum Cls { CL_APPLY0 = 0, CL_RESID, CL_DGSU, CL_PFOWN, CL_PFNBR, CL_PR, CL_RESTRICT, CL_PROLONG, NCLS };
constexpr int MAXL = 16;

struct Tab {
  int off = 0, n = 0, blocks = 0;
};

struct Carve {
  char* base;
  size_t used = 0;
  bool dry;
  template <typename T>
  T* take(size_t count) {
    used = (used + 255) & ~size_t(255);
    T* p = dry ? nullptr : (T*)(base + used);
    used += count * sizeof(T);
    return p;
  }
};

long dofs(const Geom& g) {
  return (long)(g.nx - 1) * g.ny * g.nz + (long)g.nx * (g.ny - 1) * g.nz + (long)g.nx * g.ny * (g.nz - 1) +
         (long)g.nx * g.ny * g.nz;
}

// Levels of one domain: the single-domain automatic rule (halve while every
// axis is even and stays >= 4 cells), deepened (down to >= 2 cells) while the
// coarsest system would exceed the dense-solve limit; or the explicit count.
int domain_levels(const stokes_params& p) {
  if (p.levels > 0) return p.levels;
  int L = count_levels(p.nx, p.ny, p.nz, 4);
  const int Lmax = count_levels(p.nx, p.ny, p.nz, 2);
  while (L < Lmax && dofs(make_geom(p.nx, p.ny, p.nz, p.h, p.eta, p.gamma, L - 1)) > 2500) ++L;
  return L;
}

int validate_batch(int n, const stokes_params* p) {
  if (n < 1 || !p) return STOKES_EINVAL;
  for (int i = 0; i < n; ++i) {
    const stokes_params& q = p[i];
    if (q.nx < 2 || q.ny < 2 || q.nz < 2 || !(q.h > 0) || !(q.eta > 0) || !(q.gamma > 0) || q.labels) return STOKES_EINVAL;
    if (q.nu < 1 || q.n_boundary < 1) return STOKES_EINVAL;
    if (q.smoother != STOKES_SMOOTHER_SPLIT && q.smoother != STOKES_SMOOTHER_SYMMETRIC) return STOKES_EINVAL;
    if (q.smoother == STOKES_SMOOTHER_SYMMETRIC && q.nu % 2) return STOKES_EINVAL;
    if (q.vcycle_precision != 64 && q.vcycle_precision != 32) return STOKES_EINVAL;
    // batches run the paper's V-cycle with the 8-colour multiplicative Vanka
    if (q.vanka != STOKES_VANKA_MULT8 || q.cycle != 1) return STOKES_EINVAL;
    // the smoothing schedule runs level-synchronously: one schedule for the batch
    if (q.nu != p[0].nu || q.n_boundary != p[0].n_boundary || q.smoother != p[0].smoother ||
        q.vcycle_precision != p[0].vcycle_precision)
      return STOKES_EINVAL;
    const int L = domain_levels(q);
    if (L < 1 || L > count_levels(q.nx, q.ny, q.nz, 2) || L > MAXL) return STOKES_EINVAL;
    const Geom g0 = make_geom(q.nx, q.ny, q.nz, q.h, q.eta, q.gamma, 0);
    if ((long)g0.field * 4 >= (1L << 31) - 1024) return STOKES_EINVAL;
    if (dofs(make_geom(q.nx, q.ny, q.nz, q.h, q.eta, q.gamma, L - 1)) > 2500) return STOKES_EINVAL;
  }
  return STOKES_OK;
}

}  // namespace

struct stokes_batch {
  int D = 0, prec = 64, Lmax = 0;
  std::vector<stokes_params> prm;
  std::vector<int> L;
  hipStream_t stream = nullptr, cap = nullptr;
  // per level: host and device BLev arrays (indexed by domain), participation lists
  std::vector<std::vector<BLev>> hlev;
  BLev* dlev[MAXL] = {};
  std::vector<int> all[MAXL], smooth[MAXL], coarse[MAXL];
  // batch vectors
  std::vector<long> hvoff, hvlen;
  long* voff = nullptr;
  long* vlen = nullptr;
  long vtotal = 0;
  double *s = nullptr, *t = nullptr, *q = nullptr, *dv = nullptr;
  double* partial = nullptr;
  BScal* sc = nullptr;
  int* done = nullptr;
  int* aux = nullptr;
  int* count = nullptr;
  int* hcount = nullptr;  // pinned
  BScal* hsc = nullptr;   // pinned
  // tables
  std::vector<BEnt> harena;
  BEnt* arena = nullptr;
  Tab tcls[NCLS][MAXL][NBX];
  Tab tvec, tfield, tzero[MAXL], tcoarse[MAXL], tvanka[MAXL][4], tvapply[MAXL][4], tband[MAXL], tpp[MAXL][8];
  bool vpp[MAXL] = {};  // level runs the two-copy Vanka passes (else delta and apply launches)
  void* vdelta = nullptr;
  Tab tsweep[MAXL];  // boxes whose Vanka step on the level runs in one workgroup
  int bx[NCLS][MAXL];
  int chunk_first = 10, chunk = 2;
  // graphs, keyed by (b, x)
  struct G {
    const double* b = nullptr;
    double* x = nullptr;
    hipGraphExec_t first = nullptr, more = nullptr;
  };
  std::vector<G> graphs;
  hipStream_t ks = nullptr;

  const BEnt* tab(const Tab& t) const { return arena + t.off; }
};

namespace {

void drop_graphs(stokes_batch* c) {
  for (auto& g : c->graphs) {
    if (g.first) (void)hipGraphExecDestroy(g.first);
    if (g.more) (void)hipGraphExecDestroy(g.more);
  }
  c->graphs.clear();
}

Tab add_table(stokes_batch* c, const std::vector<int>& doms, const std::function<int(int)>& nblocks) {
  Tab t;
  t.off = (int)c->harena.size();
  int acc = 0;
  for (int d : doms) {
    const int nb = nblocks(d);
    if (nb <= 0) continue;
    c->harena.push_back(BEnt{d, acc});
    acc += nb;
    ++t.n;
  }
  c->harena.push_back(BEnt{-1, acc});  // closing entry
  t.blocks = acc;
  return t;
}

// Lay out (or size) everything; host tables are built as a side effect.
void carve(stokes_batch* c, Carve& cv) {
  const int D = c->D;
  c->prec = c->prm[0].vcycle_precision;
  const size_t es = c->prec == 32 ? sizeof(float) : sizeof(double);
  c->Lmax = 0;
  c->L.resize(D);
  for (int d = 0; d < D; ++d) {
    c->L[d] = domain_levels(c->prm[d]);
    c->Lmax = std::max(c->Lmax, c->L[d]);
  }
  c->hlev.assign(c->Lmax, std::vector<BLev>(D));
  for (int l = 0; l < c->Lmax; ++l) {
    c->all[l].clear();
    c->smooth[l].clear();
    c->coarse[l].clear();
  }
  c->hvoff.assign(D, 0);
  c->hvlen.assign(D, 0);
  long off = 0;
  for (int d = 0; d < D; ++d) {
    const stokes_params& p = c->prm[d];
    for (int l = 0; l < c->L[d]; ++l) {
      BLev& b = c->hlev[l][d];
      b = BLev{};
      b.g = make_geom(p.nx, p.ny, p.nz, p.h, p.eta, p.gamma, l);
      if (l + 1 < c->L[d]) b.gc = make_geom(p.nx, p.ny, p.nz, p.h, p.eta, p.gamma, l + 1);
      c->all[l].push_back(d);
      (l + 1 < c->L[d] ? c->smooth[l] : c->coarse[l]).push_back(d);
    }
    c->hvoff[d] = off;
    c->hvlen[d] = 4L * c->hlev[0][d].g.field;
    off += (c->hvlen[d] + 1023) / 1024 * 1024;
  }
  c->vtotal = off;
  c->s = cv.take<double>(off);
  c->t = cv.take<double>(off);
  c->q = cv.take<double>(off);
  c->dv = cv.take<double>(off);
  c->voff = cv.take<long>(D);
  c->vlen = cv.take<long>(D);
  c->sc = cv.take<BScal>(D);
  c->done = cv.take<int>(D);
  c->aux = cv.take<int>(D);
  c->count = cv.take<int>(1);
  // per-domain level data
  long vmax = 1;
  for (int l = 0; l < c->Lmax; ++l) {
    long vsum[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // cells per class over the boxes (eight lanes each)
    long psum[4] = {0, 0, 0, 0};              // their corrections per pair
    for (int d : c->all[l]) {
      BLev& b = c->hlev[l][d];
      const long tot = 4L * b.g.field;
      if (l > 0 || c->prec == 32) {
        b.x = cv.take<char>(tot * es);
        b.b = cv.take<char>(tot * es);
      } else if (!cv.dry) {
        b.x = c->t + c->hvoff[d];
        b.b = c->s + c->hvoff[d];
      }
      if (l + 1 < c->L[d]) {
        b.r = cv.take<char>(tot * es);
        b.dscr = cv.take<char>((size_t)b.g.field * es);
        b.kinv = cv.take<char>(64 * 64 * es);
        std::vector<int> cells[8];
        vanka_cells(b.g, cells);
        bool small = true;
        // classes q and 7-q back to back: their pair pass (vanka_pair8) reads one list
        for (int k = 0; k < 8; ++k) {
          b.nv[k] = (int)cells[k].size();
          if (k < 4)
            b.vc[k] = cv.take<int>(std::max<size_t>(cells[k].size() + cells[7 - k].size(), 1));
          else
            b.vc[k] = b.vc[7 - k] ? b.vc[7 - k] + b.nv[7 - k] : nullptr;
          small = small && b.nv[k] <= VSWEEP_MAX_CLASS;
        }
        if (!small) {
          for (int k = 0; k < 8; ++k) vsum[k] += 8L * b.nv[k];
          for (int q = 0; q < 4; ++q) {
            b.voff[q] = psum[q];
            psum[q] += 8L * (b.nv[q] + b.nv[7 - q]);
          }
        }
      } else {
        b.nc = (int)dofs(b.g);
        b.cinv = cv.take<double>((size_t)b.nc * b.nc);
        b.cdof = cv.take<int>(b.nc);
      }
    }
    // two copies where every class, summed over the boxes, fits the eight-lane size of a
    // single box's latency-bound levels; larger levels keep the delta and apply launches
    c->vpp[l] = true;
    for (int k = 0; k < 8; ++k) c->vpp[l] = c->vpp[l] && vsum[k] / 8 <= VANKA_LANES_MAX;
    for (int q = 0; q < 4; ++q) vmax = std::max(vmax, psum[q]);
    for (int d : c->all[l]) {
      BLev& b = c->hlev[l][d];
      if (c->vpp[l] && l + 1 < c->L[d]) {
        bool small = true;
        for (int k = 0; k < 8; ++k) small = small && b.nv[k] <= VSWEEP_MAX_CLASS;
        if (!small) b.alt = cv.take<char>(4L * b.g.field * es);
      }
    }
  }
  c->vdelta = cv.take<char>(vmax * es);
  for (int l = 0; l < c->Lmax; ++l) {
    for (int d : c->all[l]) {
      BLev& b = c->hlev[l][d];
      if (l + 1 < c->L[d]) {
        b.xc = nullptr;  // filled below once the next level is carved
        b.bc = nullptr;
      }
    }
  }
  for (int l = 0; l + 1 < c->Lmax; ++l)
    for (int d : c->smooth[l]) {
      c->hlev[l][d].xc = c->hlev[l + 1][d].x;
      c->hlev[l][d].bc = c->hlev[l + 1][d].b;
    }
  for (int l = 0; l < c->Lmax; ++l) c->dlev[l] = cv.take<BLev>(D);
  // tables
  c->harena.clear();
  std::vector<int> doms(D);
  for (int d = 0; d < D; ++d) doms[d] = d;
  long maxblk = 1;
  auto note = [&](const Tab& t) { maxblk = std::max<long>(maxblk, t.blocks); };
  c->tvec = add_table(c, doms, [&](int d) { return (int)((c->hvlen[d] + 4 * BS - 1) / (4 * BS)); });
  note(c->tvec);
  c->tfield = add_table(c, doms, [&](int d) { return (c->hlev[0][d].g.field + BS - 1) / BS; });
  note(c->tfield);
  for (int v = 0; v < NBX; ++v) {
    auto dslot = [&](int l, int d) -> int {  // DGS classes: row packs, flat
      const Geom& g = c->hlev[l][d].g;
      const int V = c->prec == 32 ? 4 : 2;
      return flat_blocks(g, (((g.sy + 1) >> 1) + V - 1) / V);
    };
    auto cslot = [&](int l, int d) -> int {
      const Geom& g = c->hlev[l][d].gc;
      switch (v) {
        case 0: return tile_blocks<32>(g, g.sy);
        case 1: return tile_blocks<64>(g, g.sy);
        case 2: return tile_blocks<128>(g, g.sy);
        default: return tile_blocks<256>(g, g.sy);
      }
    };
    // operator passes: slot packs laid out flat (FP64 packs of 2 at level 0; V-cycle precision below)
    auto apack = [&](int l, int d, int V) -> int {
      const Geom& g = c->hlev[l][d].g;
      return flat_blocks(g, 2 * ((((g.sy + 1) >> 1) + V - 1) / V));
    };
    c->tcls[CL_APPLY0][0][v] = add_table(c, doms, [&](int d) { return apack(0, d, 2); });
    note(c->tcls[CL_APPLY0][0][v]);
    for (int l = 0; l < c->Lmax; ++l) {
      const std::vector<int>& S = c->smooth[l];
      c->tcls[CL_RESID][l][v] = add_table(c, S, [&](int d) { return apack(l, d, c->prec == 32 ? 4 : 2); });
      // prolongation: one thread per pair of coarse cells, flat
      c->tcls[CL_PROLONG][l][v] = add_table(c, S, [&](int d) {
        const Geom& gc = c->hlev[l][d].gc;
        return flat_blocks(gc, (gc.nx + 1) >> 1);
      });
      c->tcls[CL_RESTRICT][l][v] = add_table(c, S, [&](int d) { return cslot(l, d); });
      // DGS classes: row packs of 16 bytes (V cells)
      for (int k : {CL_DGSU, CL_PFOWN, CL_PFNBR, CL_PR})
        c->tcls[k][l][v] = add_table(c, S, [&](int d) { return dslot(l, d); });
    }
  }
  for (int l = 0; l < c->Lmax; ++l) {
    c->tzero[l] = add_table(c, c->all[l], [&](int d) {
      return (int)((4L * c->hlev[l][d].g.field + 4 * BS - 1) / (4 * BS));
    });
    c->tcoarse[l] = add_table(c, c->coarse[l], [&](int d) { return (c->hlev[l][d].nc + 3) / 4; });
    // small boxes of the level: the whole Vanka step in one workgroup each;
    // the others one launch per class pass
    auto small = [&](int d) {
      for (int k = 0; k < 8; ++k)
        if (c->hlev[l][d].nv[k] > VSWEEP_MAX_CLASS) return false;
      return true;
    };
    c->tsweep[l] = add_table(c, c->smooth[l], [&](int d) { return small(d) ? 1 : 0; });
    for (int q = 0; q < 4; ++q) {
      auto blocks = [&](int d) {
        const BLev& b = c->hlev[l][d];
        return c->vpp[l] || small(d) ? 0 : (8 * (b.nv[q] + b.nv[7 - q]) + BS - 1) / BS;
      };
      c->tvanka[l][q] = add_table(c, c->smooth[l], blocks);
      c->tvapply[l][q] = add_table(c, c->smooth[l], blocks);
    }
    // two-copy passes: the band copy, then pass p of pair q with the previous pair qp
    c->tband[l] = add_table(c, c->smooth[l], [&](int d) {
      const Geom& g = c->hlev[l][d].g;
      if (!c->vpp[l] || small(d)) return 0;
      const long n = (g.nx < 8 || g.ny < 8 || g.nz < 8) ? 4L * g.field : vanka_band_slots(g);
      return (int)((n + BS - 1) / BS);
    });
    for (int pass = 0; pass < VANKA_PASSES8; ++pass) {
      const int q = vanka_pair8(pass), qp = vanka_pair8_prev(pass);
      c->tpp[l][pass] = add_table(c, c->smooth[l], [&](int d) {
        if (!c->vpp[l] || small(d)) return 0;
        const BLev& b = c->hlev[l][d];
        const int lanes = (8 * (b.nv[q] + b.nv[7 - q]) + 63) / 64 * 64 + (qp >= 0 ? 8 * (b.nv[qp] + b.nv[7 - qp]) : 0);
        return (lanes + BS - 1) / BS;
      });
    }
  }
  c->partial = cv.take<double>(2 * maxblk);
  c->arena = cv.take<BEnt>(c->harena.size());
}

// ------------------------------------------------------------ launches

inline int grid_of(const Tab& t) { return t.blocks; }

#define BX_CASE(VAR, ...)                   \
  switch (VAR) {                            \
    case 0: { constexpr int BXT = 32; __VA_ARGS__; } break;   \
    case 1: { constexpr int BXT = 64; __VA_ARGS__; } break;   \
    case 2: { constexpr int BXT = 128; __VA_ARGS__; } break;  \
    default: { constexpr int BXT = 256; __VA_ARGS__; } break; \
  }

template <typename T>
void l_resid(stokes_batch* c, int l, int v) {
  const Tab& t = c->tcls[CL_RESID][l][v];
  if (!t.n) return;
  BX_CASE(v, kb_resid<T, BXT><<<t.blocks, BS, 0, c->ks>>>(c->tab(t), t.n, c->dlev[l], c->done))
}
// arg: the colour (CL_DGSU), the forward launch t = 0..3 (CL_PFOWN; CL_PFNBR is
// launch 4, the last neighbour update) or the reverse stage (CL_PR)
template <typename T>
void l_dgs(stokes_batch* c, int cls, int l, int v, int arg) {
  const Tab& t = c->tcls[cls][l][v];
  if (!t.n) return;
  const BEnt* tb = c->tab(t);
  BLev* lv = c->dlev[l];
  switch (cls) {
    case CL_DGSU: BX_CASE(v, kb_dgs_u<T, BXT><<<t.blocks, BS, 0, c->ks>>>(tb, t.n, lv, c->done, arg)) break;
    case CL_PFOWN: BX_CASE(v, kb_dgs_pf<T, BXT><<<t.blocks, BS, 0, c->ks>>>(tb, t.n, lv, c->done, arg)) break;
    case CL_PFNBR: BX_CASE(v, kb_dgs_pf<T, BXT><<<t.blocks, BS, 0, c->ks>>>(tb, t.n, lv, c->done, 4)) break;
    default: BX_CASE(v, kb_dgs_pr<T, BXT><<<t.blocks, BS, 0, c->ks>>>(tb, t.n, lv, c->done, arg)) break;
  }
}
template <typename T>
void l_restrict(stokes_batch* c, int l, int v) {
  const Tab& t = c->tcls[CL_RESTRICT][l][v];
  if (!t.n) return;
  BX_CASE(v, kb_restrict<T, BXT><<<t.blocks, BS, 0, c->ks>>>(c->tab(t), t.n, c->dlev[l], c->done))
}
template <typename T>
void l_prolong(stokes_batch* c, int l, int v) {
  const Tab& t = c->tcls[CL_PROLONG][l][v];
  if (!t.n) return;
  BX_CASE(v, kb_prolong<T, BXT><<<t.blocks, BS, 0, c->ks>>>(c->tab(t), t.n, c->dlev[l], c->done))
}

template <typename T>
void b_vanka_symmetric(stokes_batch* c, int l) {
  const Tab& ts = c->tsweep[l];
  if (ts.n) kb_vanka_sweep<T><<<ts.blocks, VSWEEP_BS, 0, c->ks>>>(c->tab(ts), ts.n, c->dlev[l], c->done);
  if (!c->vpp[l]) {  // the other boxes: residual and correction launches per pair pass
    for (int pass = 0; pass < VANKA_PASSES8; ++pass) {
      const int q = vanka_pair8(pass);
      const Tab& t = c->tvanka[l][q];
      const Tab& ta = c->tvapply[l][q];
      if (!t.n) continue;
      kb_vanka_delta<T><<<t.blocks, BS, 0, c->ks>>>(c->tab(t), t.n, c->dlev[l], c->done, q, (T*)c->vdelta);
      kb_vanka_apply<T><<<ta.blocks, BS, 0, c->ks>>>(c->tab(ta), ta.n, c->dlev[l], c->done, q,
                                                     (const T*)c->vdelta);
    }
    return;
  }
  // or two copies of the state, one launch per pair pass; the 8 passes end in x
  const Tab& tb = c->tband[l];
  if (!tb.n) return;
  kb_vanka_band<T><<<tb.blocks, BS, 0, c->ks>>>(c->tab(tb), tb.n, c->dlev[l], c->done);
  for (int pass = 0; pass < VANKA_PASSES8; ++pass) {
    const Tab& t = c->tpp[l][pass];
    if (!t.n) continue;
    kb_vanka_pp<T><<<t.blocks, BS, 0, c->ks>>>(c->tab(t), t.n, c->dlev[l], c->done, vanka_pair8(pass),
                                               vanka_pair8_prev(pass), pass & 1);
  }
}

// Forward sweep: velocities red, black; the pressure stages in five launches
// (packed_kernels.hpp, dgs_pf_stage_pack).
template <typename T>
void b_dgs_forward(stokes_batch* c, int l) {
  for (int col = 0; col < 2; ++col) l_dgs<T>(c, CL_DGSU, l, c->bx[CL_DGSU][l], col);
  for (int t = 0; t < 4; ++t) l_dgs<T>(c, CL_PFOWN, l, c->bx[CL_PFOWN][l], t);
  l_dgs<T>(c, CL_PFNBR, l, c->bx[CL_PFNBR][l], 4);
}

// Reverse sweep: pressure stages 3..0, then velocities black, red.
template <typename T>
void b_dgs_reverse(stokes_batch* c, int l) {
  for (int st = 3; st >= 0; --st) l_dgs<T>(c, CL_PR, l, c->bx[CL_PR][l], st);
  for (int col = 1; col >= 0; --col) l_dgs<T>(c, CL_DGSU, l, c->bx[CL_DGSU][l], col);
}

enum Interior { INT_SYMMETRIC, INT_REVERSE, INT_FORWARD };

template <typename T>
void b_smooth(stokes_batch* c, int l, Interior kind, int sweeps) {
  const stokes_params& p = c->prm[0];
  for (int i = 0; i < p.n_boundary; ++i) b_vanka_symmetric<T>(c, l);
  for (int i = 0; i < sweeps; ++i) {
    if (kind != INT_FORWARD) {
      if (kind == INT_SYMMETRIC) b_dgs_forward<T>(c, l);
      b_dgs_reverse<T>(c, l);
    } else {
      b_dgs_forward<T>(c, l);
    }
  }
  for (int i = 0; i < p.n_boundary; ++i) b_vanka_symmetric<T>(c, l);
}

template <typename T>
void b_presmooth(stokes_batch* c, int l) {
  const stokes_params& p = c->prm[0];
  if (p.smoother == STOKES_SMOOTHER_SYMMETRIC) {
    for (int i = 0; i < p.nu / 2; ++i) b_smooth<T>(c, l, INT_SYMMETRIC, 1);
  } else {
    b_smooth<T>(c, l, INT_REVERSE, p.nu);
  }
}

template <typename T>
void b_postsmooth(stokes_batch* c, int l) {
  const stokes_params& p = c->prm[0];
  if (p.smoother == STOKES_SMOOTHER_SYMMETRIC) {
    for (int i = 0; i < p.nu / 2; ++i) b_smooth<T>(c, l, INT_SYMMETRIC, 1);
  } else {
    b_smooth<T>(c, l, INT_FORWARD, p.nu);
  }
}

// Level l of the V-cycle of every domain that has it (Alg. 1): the domains
// whose coarsest level is l solve there, the others smooth, restrict, recurse,
// prolong and smooth again.
template <typename T>
void b_vcycle(stokes_batch* c, int l) {
  const Tab& z = c->tzero[l];
  if (z.n) kb_zero_level<T><<<z.blocks, BS, 0, c->ks>>>(c->tab(z), z.n, c->dlev[l], c->done);
  const Tab& co = c->tcoarse[l];
  if (co.n) kb_coarse<T><<<co.blocks, BS, 0, c->ks>>>(c->tab(co), co.n, c->dlev[l], c->done);
  if (c->smooth[l].empty()) return;
  b_presmooth<T>(c, l);
  l_resid<T>(c, l, c->bx[CL_RESID][l]);
  l_restrict<T>(c, l, c->bx[CL_RESTRICT][l]);
  b_vcycle<T>(c, l + 1);
  l_prolong<T>(c, l, c->bx[CL_PROLONG][l]);
  b_postsmooth<T>(c, l);
}

// t = W s for every active domain.  FP32 V-cycle inside the iterations: s's
// update has already written the float right-hand sides, and the SQMR passes
// read the float result where it lies (fused = true); else both conversions.
void b_precondition(stokes_batch* c, bool fused = false) {
  if (c->prec == 64) {
    b_vcycle<double>(c, 0);
    return;
  }
  const Tab& tv = c->tvec;
  if (!fused)
    kb_convert<double, float, true><<<tv.blocks, BS, 0, c->ks>>>(c->tab(tv), tv.n, c->done, c->voff, c->vlen,
                                                                 c->dlev[0], c->s, (float*)nullptr);
  b_vcycle<float>(c, 0);
  if (!fused)
    kb_convert<float, double, false><<<tv.blocks, BS, 0, c->ks>>>(c->tab(tv), tv.n, c->done, c->voff, c->vlen,
                                                                  c->dlev[0], (const float*)nullptr, c->t);
}

// ----------------------------------------------------- device SQMR scalars

__global__ void kb_sq_reset(BScal* sc, int* done, int D, double rtol, int maxit) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D) return;
  BScal& s = sc[d];
  s.rho = s.tau = s.nu_prev = s.alpha = s.beta = s.cd = s.cq = 0.0;
  s.bnorm = s.relres = NAN;
  s.rtol = rtol;
  s.iters = 0;
  s.status = STOKES_OK;
  s.maxit = maxit;
  s.zero_x = 0;
  done[d] = 0;
}

__global__ void kb_sq_bnorm(BScal* sc, int* done, int D) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D || done[d]) return;
  BScal& s = sc[d];
  s.bnorm = sqrt(s.red[RED0]);
  if (!isfinite(s.bnorm)) {
    s.status = STOKES_ENONFINITE;
    done[d] = 1;
  } else if (s.bnorm == 0.0) {
    s.relres = 0.0;
    s.zero_x = 1;
    done[d] = 1;
  }
}

__global__ void kb_sq_r0(BScal* sc, int* done, int D) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D || done[d]) return;
  BScal& s = sc[d];
  s.relres = sqrt(s.red[RED0]) / s.bnorm;
  if (!isfinite(s.relres)) {
    s.status = STOKES_ENONFINITE;
    done[d] = 1;
  } else if (s.relres <= s.rtol) {
    done[d] = 1;
  } else if (s.maxit == 0) {
    s.status = STOKES_ENOCONV;
    done[d] = 1;
  }
}

__global__ void kb_sq_start(BScal* sc, const int* done, int D) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D || done[d]) return;
  BScal& s = sc[d];
  s.tau = sqrt(s.red[RED0]);
  s.rho = s.red[RED1];
  s.nu_prev = 0.0;
}

__global__ void kb_sq_alpha(BScal* sc, int* done, int D) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D || done[d]) return;
  BScal& s = sc[d];
  const double sigma = s.red[RED0];
  if (!isfinite(sigma)) {
    s.status = STOKES_ENONFINITE;
    done[d] = 1;
  } else if (sigma == 0.0) {
    s.status = STOKES_EBREAKDOWN;
    done[d] = 1;
  } else {
    s.alpha = s.rho / sigma;
  }
}

__global__ void kb_sq_nu(BScal* sc, const int* done, int D) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D || done[d]) return;
  BScal& s = sc[d];
  const double tnorm = sqrt(s.red[RED0]);
  s.red[2] = s.red[RED1];  // rho_new
  s.red[3] = tnorm;
  const double nu = tnorm / s.tau;
  const double cc = 1.0 / sqrt(1.0 + nu * nu);
  s.tau = s.tau * nu * cc;
  s.cd = cc * cc * s.nu_prev * s.nu_prev;
  s.cq = cc * cc * s.alpha;
  s.nu_prev = nu;
  s.beta = s.red[2] / s.rho;  // next direction, formed with the update (unused if the domain stops)
}

__global__ void kb_sq_check(BScal* sc, int* done, int D) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D || done[d]) return;
  BScal& s = sc[d];
  s.iters += 1;
  s.relres = sqrt(s.red[RED0]) / s.bnorm;
  if (!isfinite(s.relres) || !isfinite(s.red[3])) {
    s.status = STOKES_ENONFINITE;
    done[d] = 1;
  } else if (s.relres <= s.rtol) {
    done[d] = 1;
  } else if (s.rho == 0.0) {
    s.status = STOKES_EBREAKDOWN;
    done[d] = 1;
  } else if (s.iters >= s.maxit) {
    s.status = STOKES_ENOCONV;
    done[d] = 1;
  } else {
    s.rho = s.red[2];
  }
}

__global__ void kb_count_active(const int* done, int D, int* count) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int n = 0;
  for (int d = 0; d < D; ++d) n += done[d] ? 0 : 1;
  count[0] = n;
}

// skip[d] = 1 unless the domain converged and asks for the pressure mean removed
__global__ void kb_mean_skip(const BScal* sc, const int* flags, int D, int* skip) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D) return;
  skip[d] = (sc[d].status == STOKES_OK && flags[d]) ? 0 : 1;
}

inline int dgrid(int D) { return (D + 63) / 64; }

// ----------------------------------------------------------- solve phases

void seg(stokes_batch* c, int slot, int stride, const Tab& t, const int* skip) {
  kb_seg_reduce<<<t.n, BS, 0, c->ks>>>(c->tab(t), t.n, skip, c->partial, stride, slot, c->sc);
}

template <int MODE>
void apply0(stokes_batch* c, const double* x, const double* b, double* y) {
  const int v = c->bx[CL_APPLY0][0];
  const Tab& t = c->tcls[CL_APPLY0][0][v];
  BX_CASE(v, kb_apply_vec<MODE, BXT><<<t.blocks, BS, 0, c->ks>>>(c->tab(t), t.n, c->dlev[0], c->done, c->voff, x, b,
                                                                y, c->partial))
}

void phase_init(stokes_batch* c, const double* b, double* x) {
  const int D = c->D;
  const Tab& tf = c->tfield;
  const Tab& tv = c->tvec;
  const Tab& ta = c->tcls[CL_APPLY0][0][c->bx[CL_APPLY0][0]];
  kb_clear_ghosts<<<tf.blocks, BS, 0, c->ks>>>(c->tab(tf), tf.n, c->dlev[0], c->voff, x);
  apply0<AP_BNORM>(c, x, b, nullptr);
  seg(c, RED0, 1, ta, c->done);
  kb_sq_bnorm<<<dgrid(D), 64, 0, c->ks>>>(c->sc, c->done, D);
  kb_zero_flagged<<<tv.blocks, BS, 0, c->ks>>>(c->tab(tv), tv.n, c->voff, c->vlen, c->sc, x);
  apply0<AP_RESID>(c, x, b, c->s);
  apply0<AP_RESNORM>(c, x, b, nullptr);
  seg(c, RED0, 1, ta, c->done);
  kb_sq_r0<<<dgrid(D), 64, 0, c->ks>>>(c->sc, c->done, D);
  b_precondition(c);
  kb_dot2<<<tv.blocks, BS, 0, c->ks>>>(c->tab(tv), tv.n, c->done, c->voff, c->vlen, c->t, c->s, c->partial,
                                       (const BLev*)nullptr);
  seg(c, RED0, 2, tv, c->done);
  kb_sq_start<<<dgrid(D), 64, 0, c->ks>>>(c->sc, c->done, D);
  kb_init_qd<<<tv.blocks, BS, 0, c->ks>>>(c->tab(tv), tv.n, c->done, c->voff, c->vlen, c->q, c->dv, c->t);
}

void phase_iteration(stokes_batch* c, const double* b, double* x) {
  const int D = c->D;
  const Tab& tv = c->tvec;
  const Tab& ta = c->tcls[CL_APPLY0][0][c->bx[CL_APPLY0][0]];
  apply0<AP_APPLY_DOT>(c, c->q, nullptr, c->t);
  seg(c, RED0, 1, ta, c->done);
  kb_sq_alpha<<<dgrid(D), 64, 0, c->ks>>>(c->sc, c->done, D);
  const BLev* l0 = c->prec == 32 ? c->dlev[0] : nullptr;  // FP32 V-cycle: its float level-0 vectors
  kb_axpy_neg<<<tv.blocks, BS, 0, c->ks>>>(c->tab(tv), tv.n, c->done, c->voff, c->vlen, c->sc, c->s, c->t, l0);
  b_precondition(c, l0 != nullptr);
  kb_dot2<<<tv.blocks, BS, 0, c->ks>>>(c->tab(tv), tv.n, c->done, c->voff, c->vlen, c->t, c->s, c->partial, l0);
  seg(c, RED0, 2, tv, c->done);
  kb_sq_nu<<<dgrid(D), 64, 0, c->ks>>>(c->sc, c->done, D);
  kb_update_dxq<<<tv.blocks, BS, 0, c->ks>>>(c->tab(tv), tv.n, c->done, c->voff, c->vlen, c->sc, c->dv, c->q, x,
                                             c->t, l0);
  apply0<AP_RESNORM>(c, x, b, nullptr);
  seg(c, RED0, 1, ta, c->done);
  kb_sq_check<<<dgrid(D), 64, 0, c->ks>>>(c->sc, c->done, D);
}

// capture `iters` iterations (after the set-up phase when `with_init`) into one graph
int capture(stokes_batch* c, const double* b, double* x, bool with_init, int iters, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return STOKES_EDEVICE;
  c->ks = c->cap;
  if (with_init) phase_init(c, b, x);
  for (int i = 0; i < iters; ++i) phase_iteration(c, b, x);
  c->ks = c->stream;
  const hipError_t e1 = hipStreamEndCapture(c->cap, &g);
  if (e1 != hipSuccess || !g) return STOKES_EDEVICE;
  const hipError_t e2 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e2 == hipSuccess ? STOKES_OK : STOKES_EDEVICE;
}

}  // namespace

extern "C" {

int stokes_batch_workspace_bytes(int32_t n, const stokes_params* p, size_t* bytes) {
  if (!bytes) return STOKES_EINVAL;
  const int v = validate_batch(n, p);
  if (v != STOKES_OK) return v;
  stokes_batch c;
  c.D = n;
  c.prm.assign(p, p + n);
  Carve cv{nullptr, 0, true};
  carve(&c, cv);
  *bytes = cv.used + 256;
  return STOKES_OK;
}

int stokes_batch_setup(int32_t n, const stokes_params* p, void* workspace, size_t bytes, void* hip_stream,
                       stokes_batch** out) {
  if (!out || !workspace || ((uintptr_t)workspace & 255)) return STOKES_EINVAL;
  size_t need = 0;
  const int v = stokes_batch_workspace_bytes(n, p, &need);
  if (v != STOKES_OK) return v;
  if (bytes < need) return STOKES_EINVAL;
  stokes_batch* c = new stokes_batch();
  c->D = n;
  c->prm.assign(p, p + n);
  c->stream = (hipStream_t)hip_stream;
  c->ks = c->stream;
  Carve cv{(char*)workspace, 0, false};
  carve(c, cv);
  for (int k = 0; k < NCLS; ++k)
    for (int l = 0; l < MAXL; ++l) c->bx[k][l] = 1;  // 64-wide tiles until tuned
  auto fail = [&](int code) {
    stokes_batch_destroy(c);
    return code;
  };
  if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) return fail(STOKES_EDEVICE);
  if (hipHostMalloc((void**)&c->hcount, sizeof(int)) != hipSuccess) return fail(STOKES_EDEVICE);
  if (hipHostMalloc((void**)&c->hsc, sizeof(BScal) * n) != hipSuccess) return fail(STOKES_EDEVICE);
  // dense inverses of the coarsest systems: independent per box, O(n^3) each,
  // so they are formed on host threads
  std::vector<std::vector<int>> cdofs(n);
  std::vector<std::vector<double>> cinvs(n);
  std::vector<char> cok(n, 0);
  {
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned w = 0; w < hw; ++w)
      pool.emplace_back([&, w] {
        for (int d = (int)w; d < n; d += (int)hw) {
          const BLev& b = c->hlev[c->L[d] - 1][d];
          cok[d] = coarse_inverse(b.g, cdofs[d], cinvs[d]) ? 1 : 0;
        }
      });
    for (auto& th : pool) th.join();
  }
  // upload: Vanka inverses, cells, coarse inverses, level tables, batch offsets
  const int prec = c->prec;
  std::vector<double> kd;
  std::vector<float> kf;
  for (int l = 0; l < c->Lmax; ++l)
    for (int d : c->all[l]) {
      BLev& b = c->hlev[l][d];
      if (l + 1 < c->L[d]) {
        if (!vanka_inverses(b.g, kd)) return fail(STOKES_EINVAL);
        if (prec == 32) {
          kf.assign(kd.begin(), kd.end());
          if (hipMemcpy((void*)b.kinv, kf.data(), kf.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
            return fail(STOKES_EDEVICE);
        } else if (hipMemcpy((void*)b.kinv, kd.data(), kd.size() * sizeof(double), hipMemcpyHostToDevice) !=
                   hipSuccess) {
          return fail(STOKES_EDEVICE);
        }
        std::vector<int> cells[8];
        vanka_cells(b.g, cells);
        for (int k = 0; k < 8; ++k)
          if (!cells[k].empty() &&
              hipMemcpy((void*)b.vc[k], cells[k].data(), cells[k].size() * sizeof(int), hipMemcpyHostToDevice) !=
                  hipSuccess)
            return fail(STOKES_EDEVICE);
      } else {
        if (!cok[d]) return fail(STOKES_EINVAL);
        if (hipMemcpy((void*)b.cinv, cinvs[d].data(), cinvs[d].size() * sizeof(double), hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy((void*)b.cdof, cdofs[d].data(), cdofs[d].size() * sizeof(int), hipMemcpyHostToDevice) !=
                hipSuccess)
          return fail(STOKES_EDEVICE);
        std::vector<double>().swap(cinvs[d]);
      }
    }
  for (int l = 0; l < c->Lmax; ++l)
    if (hipMemcpy(c->dlev[l], c->hlev[l].data(), sizeof(BLev) * n, hipMemcpyHostToDevice) != hipSuccess)
      return fail(STOKES_EDEVICE);
  if (hipMemcpy(c->arena, c->harena.data(), sizeof(BEnt) * c->harena.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->voff, c->hvoff.data(), sizeof(long) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->vlen, c->hvlen.data(), sizeof(long) * n, hipMemcpyHostToDevice) != hipSuccess)
    return fail(STOKES_EDEVICE);
  // the batch vectors start from zero (padding between domains stays zero)
  for (double* v : {c->s, c->t, c->q, c->dv})
    if (hipMemset(v, 0, sizeof(double) * c->vtotal) != hipSuccess) return fail(STOKES_EDEVICE);
  if (hipDeviceSynchronize() != hipSuccess) return fail(STOKES_EDEVICE);
  *out = c;
  return STOKES_OK;
}

int stokes_batch_layout(const stokes_batch* c, int32_t domain, int64_t* offset, stokes_layout_t* out) {
  if (!c || !offset || !out || domain < 0 || domain >= c->D) return STOKES_EINVAL;
  const Geom& g = c->hlev[0][domain].g;
  *offset = c->hvoff[domain];
  out->nx = g.nx;
  out->ny = g.ny;
  out->nz = g.nz;
  out->sy = g.sy;
  out->sz = g.sz;
  for (int f = 0; f < 4; ++f) out->off[f] = (int64_t)f * g.field;
  out->field = g.field;
  out->total = 4L * g.field;
  out->n_dofs = dofs(g);
  out->levels = c->L[domain];
  return STOKES_OK;
}

int stokes_batch_size(const stokes_batch* c, int64_t* total) {
  if (!c || !total) return STOKES_EINVAL;
  *total = c->vtotal;
  return STOKES_OK;
}

int stokes_batch_set_chunks(stokes_batch* c, int32_t first, int32_t later) {
  if (!c || first < 0 || later < 1) return STOKES_EINVAL;
  c->chunk_first = first;
  c->chunk = later;
  drop_graphs(c);
  return STOKES_OK;
}

int stokes_batch_autotune(stokes_batch* c, int32_t* choices) {
  if (!c) return STOKES_EINVAL;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return STOKES_EDEVICE;
  // every kernel class of every level on the batch's own buffers (their
  // contents are irrelevant: each solve starts by overwriting them)
  int rc = STOKES_OK;
  if (hipMemsetAsync(c->done, 0, sizeof(int) * c->D, c->stream) != hipSuccess) rc = STOKES_EDEVICE;
  c->ks = c->stream;
  for (int k = 0; k < NCLS && rc == STOKES_OK; ++k)
    for (int l = 0; l < c->Lmax && rc == STOKES_OK; ++l) {
      if (k == CL_APPLY0 && l > 0) continue;
      if (k != CL_APPLY0 && c->smooth[l].empty()) continue;
      float best = 1e30f;
      int bestv = c->bx[k][l];
      for (int v = 0; v < NBX; ++v) {
        c->bx[k][l] = v;
        float ms = 0.f;
        for (int rep = 0; rep < 4; ++rep) {
          (void)hipEventRecord(e0, c->stream);
          if (c->prec == 32) {
            switch (k) {
              case CL_APPLY0: apply0<AP_RESNORM>(c, c->t, c->s, nullptr); break;
              case CL_RESID: l_resid<float>(c, l, v); break;
              case CL_RESTRICT: l_restrict<float>(c, l, v); break;
              case CL_PROLONG: l_prolong<float>(c, l, v); break;
              default: l_dgs<float>(c, k, l, v, rep & 1); break;
            }
          } else {
            switch (k) {
              case CL_APPLY0: apply0<AP_RESNORM>(c, c->t, c->s, nullptr); break;
              case CL_RESID: l_resid<double>(c, l, v); break;
              case CL_RESTRICT: l_restrict<double>(c, l, v); break;
              case CL_PROLONG: l_prolong<double>(c, l, v); break;
              default: l_dgs<double>(c, k, l, v, rep & 1); break;
            }
          }
          (void)hipEventRecord(e1, c->stream);
          if (hipEventSynchronize(e1) != hipSuccess) {
            rc = STOKES_EDEVICE;
            break;
          }
          float t = 0.f;
          (void)hipEventElapsedTime(&t, e0, e1);
          if (rep > 0) ms += t;  // the first run warms the caches
        }
        if (ms < best) {
          best = ms;
          bestv = v;
        }
      }
      c->bx[k][l] = bestv;
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (choices)
    for (int k = 0; k < NCLS; ++k)
      for (int l = 0; l < MAXL; ++l) {
        const bool used = k == CL_APPLY0 ? l == 0 : (l < c->Lmax && !c->smooth[l].empty());
        choices[k * MAXL + l] = used ? BXV[c->bx[k][l]] : 0;
      }
  drop_graphs(c);
  if (hipGetLastError() != hipSuccess) rc = STOKES_EDEVICE;
  return rc;
}

int stokes_batch_solve(stokes_batch* c, const double* b, double* x, double rtol, int32_t maxit, stokes_info* info) {
  if (!c || !b || !x || b == x || maxit < 0 || !(rtol >= 0)) return STOKES_EINVAL;
  const int D = c->D;
  stokes_batch::G* gr = nullptr;
  for (auto& g : c->graphs)
    if (g.b == b && g.x == x) gr = &g;
  if (!gr) {
    if (c->graphs.size() >= 4) drop_graphs(c);
    c->graphs.push_back(stokes_batch::G{b, x, nullptr, nullptr});
    gr = &c->graphs.back();
    if (capture(c, b, x, true, c->chunk_first, &gr->first) != STOKES_OK ||
        capture(c, b, x, false, c->chunk, &gr->more) != STOKES_OK) {
      drop_graphs(c);
      return STOKES_EDEVICE;
    }
  }
  kb_sq_reset<<<dgrid(D), 64, 0, c->stream>>>(c->sc, c->done, D, rtol, maxit);
  if (hipGraphLaunch(gr->first, c->stream) != hipSuccess) return STOKES_EDEVICE;
  int launched = c->chunk_first;
  for (;;) {
    kb_count_active<<<1, 64, 0, c->stream>>>(c->done, D, c->count);
    if (hipMemcpyAsync(c->hcount, c->count, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return STOKES_EDEVICE;
    if (*c->hcount == 0 || launched >= maxit) break;
    if (hipGraphLaunch(gr->more, c->stream) != hipSuccess) return STOKES_EDEVICE;
    launched += c->chunk;
  }
  // pressure mean of the converged domains that ask for it
  std::vector<int> flags(D);
  for (int d = 0; d < D; ++d) flags[d] = (c->prm[d].flags & STOKES_FLAG_REMOVE_MEAN) ? 1 : 0;
  if (hipMemcpyAsync(c->aux, flags.data(), sizeof(int) * D, hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return STOKES_EDEVICE;
  kb_mean_skip<<<dgrid(D), 64, 0, c->stream>>>(c->sc, c->aux, D, c->aux);
  const Tab& tf = c->tfield;
  kb_sum_p<<<tf.blocks, BS, 0, c->stream>>>(c->tab(tf), tf.n, c->dlev[0], c->aux, c->voff, x, c->partial);
  kb_seg_reduce<<<tf.n, BS, 0, c->stream>>>(c->tab(tf), tf.n, c->aux, c->partial, 1, RED0, c->sc);
  kb_shift_p<<<tf.blocks, BS, 0, c->stream>>>(c->tab(tf), tf.n, c->dlev[0], c->aux, c->voff, c->sc, x);
  if (hipMemcpyAsync(c->hsc, c->sc, sizeof(BScal) * D, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess || hipGetLastError() != hipSuccess)
    return STOKES_EDEVICE;
  int first_bad = STOKES_OK;
  for (int d = 0; d < D; ++d) {
    const BScal& s = c->hsc[d];
    if (info) {
      info[d].iters = s.iters;
      info[d].status = s.status;
      info[d].relres = s.relres;
      info[d].bnorm = s.bnorm;
    }
    if (s.status != STOKES_OK && first_bad == STOKES_OK) first_bad = s.status;
  }
  return first_bad;
}

void stokes_batch_destroy(stokes_batch* c) {
  if (!c) return;
  drop_graphs(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->hcount) (void)hipHostFree(c->hcount);
  if (c->hsc) (void)hipHostFree(c->hsc);
  delete c;
}

}  // extern "C"
