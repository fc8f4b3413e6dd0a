/*
 * Plain CPU oracle for the ES-PIC particle step (arXiv:1604.07713).
 * THIS IS TEST INFRASTRUCTURE: only tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU library.
 *
 * Build: g++ -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (no FMA
 * contraction, so FP32 instantiations are an IEEE mirror of the GPU's FP32
 * arithmetic and FP64 ones of its FP64 arithmetic).
 *
 * What each part follows, and what pins it (tests/test_oracle_*.py):
 *   Philox4x32-10 / 4x64-10 (counter-based RNG of Salmon et al., SC'11):
 *       the 4x64 instantiation of the same generic round function is pinned
 *       bit-exactly to numpy.random.Philox; the 4x32 constants are the
 *       published ones (pinned by citation plus uniformity statistics).
 *   Gather/push (Sec. 3, explicit leapfrog, bilinear E from nodal values):
 *       free particle in uniform E (exact quadratic), harmonic motion in a
 *       linear field (closed-form recurrence), cold-plasma oscillation.
 *   CIC / NGP deposit (Sec. 3; no volume weighting, Sec. 3.1):
 *       exact charge sums, first moment, brute-force counts.
 *   Locate on the quadtree (Sec. 3.1): brute force over all leaves.
 *   1D Poisson (exact inverse of the tridiagonal operator, integer sums):
 *       closed-form parabola, scipy banded solver, exact rational arithmetic.
 *   2D cell-centred Poisson (FV + Jacobi CG): scipy sparse direct solve,
 *       manufactured-solution convergence.
 *   Nodal E from cell/corner potentials: exact for linear potentials on any
 *       2:1 tree.
 *   MCC null-collision (Sec. 3): event rates vs n*sigma*v (binomial 5 sigma),
 *       elastic energy loss 2m/M, isotropy moments, ionization energy balance.
 *   Births / split / merge (Sec. 4.3): exact count, weight, charge identities.
 *   Adapt (Sec. 3.1, 4.3): 2:1 balance, area sum, level bounds, idempotence;
 *       the coarsen rule on a hand-built explicit tree whose expected leaf
 *       set is written down, one sibling group per condition.
 *   Coarse-fine face coefficient of the FV operator: a linear potential
 *       across faces between levels is annihilated, and a manufactured
 *       solution converges at second order, on trees with such faces.
 *   Cell-to-node potential at hanging nodes: exact for linear cell
 *       potentials against the mean of the incident leaf centres.
 *   Merge pairing by (velocity octant, |v|^2, id): one leaf whose pairs are
 *       listed by hand.
 *   Charge density: integrates to the total charge exactly (to rounding).
 *   The tree pins are checked against planted mistakes (a copy of this file
 *       with one rule changed must fail them: tests/test_oracle_mutants.py).
 * Where the paper leaves a point open, the reading taken is stated at the
 * function that implements it.
 */
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <map>
#include <utility>
#include <vector>

namespace {

/* CODATA 2018 exact / recommended values */
const double QE = 1.602176634e-19;
const double EPS0 = 8.8541878128e-12;
const double KB = 1.380649e-23;

/* ------------------------------------------------------------------ */
/* Philox-4xW-10: the generic round of the published generator.        */
/* ------------------------------------------------------------------ */
template <class W> struct PhiloxK;
template <> struct PhiloxK<uint32_t> {
  static constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  static constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  static void mulhilo(uint32_t a, uint32_t b, uint32_t& hi, uint32_t& lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    hi = (uint32_t)(p >> 32);
    lo = (uint32_t)p;
  }
};
template <> struct PhiloxK<uint64_t> {
  static constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  static constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  static void mulhilo(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    hi = (uint64_t)(p >> 64);
    lo = (uint64_t)p;
  }
};

template <class W>
void philox10(const W ctr[4], const W key[2], W out[4]) {
  W x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  W k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {           /* key schedule: Weyl sequence */
      k0 += PhiloxK<W>::W0;
      k1 += PhiloxK<W>::W1;
    }
    W hi0, lo0, hi1, lo1;
    PhiloxK<W>::mulhilo(PhiloxK<W>::M0, x0, hi0, lo0);
    PhiloxK<W>::mulhilo(PhiloxK<W>::M1, x2, hi1, lo1);
    W y0 = hi1 ^ x1 ^ k0;
    W y1 = lo1;
    W y2 = hi0 ^ x3 ^ k1;
    W y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Per-(particle, step) word stream: counter = (id, step, block, 0). */
struct Stream {
  uint32_t key[2];
  uint32_t id, step, block;
  uint32_t w[4];
  int pos;
  Stream(uint64_t seed, uint32_t ikey, uint32_t id_, uint32_t step_) {
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32) ^ ikey;
    id = id_; step = step_; block = 0; pos = 0;
    gen();
  }
  void gen() {
    uint32_t c[4] = {id, step, block, 0u};
    philox10<uint32_t>(c, key, w);
  }
  uint32_t next() {
    if (pos == 4) { ++block; gen(); pos = 0; }
    return w[pos++];
  }
};

/* uniform in (0,1): odd multiple of 2^-24, exact in FP32 and FP64 */
template <class T> T uniform(uint32_t r) {
  return (T)(2u * (r >> 9) + 1u) * (T)5.9604644775390625e-08;
}

/* isotropic unit vector, Marsaglia (1972) rejection on the unit disk */
template <class T> void iso_dir(Stream& st, T d[3]) {
  for (int k = 0; k < 32; ++k) {
    T a = (T)2 * uniform<T>(st.next()) - (T)1;
    T b = (T)2 * uniform<T>(st.next()) - (T)1;
    T s = a * a + b * b;
    if (s < (T)1) {
      T t = (T)2 * std::sqrt((T)1 - s);
      d[0] = a * t;
      d[1] = b * t;
      d[2] = (T)1 - (T)2 * s;
      return;
    }
  }
  d[0] = (T)0; d[1] = (T)0; d[2] = (T)1;
}

/* standard normal deviate: Irwin-Hall sum of 12 uniforms minus 6, exact in
   integers before one conversion */
template <class T> T gauss12(Stream& st) {
  int32_t S = 0;
  for (int k = 0; k < 12; ++k) S += (int32_t)(2u * (st.next() >> 9) + 1u);
  return (T)(S - 100663296) * (T)5.9604644775390625e-08;
}

/* ------------------------------------------------------------------ */
/* Quadtree (pointer form)                                              */
/* ------------------------------------------------------------------ */
struct QNode {
  int level;
  uint32_t ix, iy;
  QNode* parent;
  std::unique_ptr<QNode> kid[4];   /* SW, SE, NW, NE */
  int64_t leaf_index;
  bool is_leaf() const { return !kid[0]; }
  double h() const { return std::ldexp(1.0, -level); }
  double x0() const { return ix * h(); }
  double y0() const { return iy * h(); }
  double x1() const { return (ix + 1) * h(); }
  double y1() const { return (iy + 1) * h(); }
};

void refine_node(QNode* n) {
  for (int c = 0; c < 4; ++c) {
    n->kid[c].reset(new QNode());
    QNode* k = n->kid[c].get();
    k->level = n->level + 1;
    k->ix = 2 * n->ix + (c & 1);
    k->iy = 2 * n->iy + (c >> 1);
    k->parent = n;
    k->leaf_index = -1;
  }
}

void collect_leaves(QNode* n, std::vector<QNode*>& out) {
  if (n->is_leaf()) { n->leaf_index = (int64_t)out.size(); out.push_back(n); return; }
  for (int c = 0; c < 4; ++c) collect_leaves(n->kid[c].get(), out);
}

/* leaves whose closed box meets the closed rectangle */
void touching(QNode* n, double x0, double y0, double x1, double y1, std::vector<QNode*>& out) {
  if (n->x0() > x1 || x0 > n->x1() || n->y0() > y1 || y0 > n->y1()) return;
  if (n->is_leaf()) { out.push_back(n); return; }
  for (int c = 0; c < 4; ++c) touching(n->kid[c].get(), x0, y0, x1, y1, out);
}

QNode* locate_node(QNode* root, double sx, double sy) {
  QNode* n = root;
  while (!n->is_leaf()) {
    double hh = std::ldexp(1.0, -(n->level + 1));
    double mx = (2 * n->ix + 1) * hh, my = (2 * n->iy + 1) * hh;
    int c = (sx >= mx ? 1 : 0) | (sy >= my ? 2 : 0);
    n = n->kid[c].get();
  }
  return n;
}

uint32_t morton16(uint32_t x, uint32_t y) {
  uint32_t k = 0;
  for (int b = 0; b < 16; ++b) {
    k |= ((x >> b) & 1u) << (2 * b);
    k |= ((y >> b) & 1u) << (2 * b + 1);
  }
  return k;
}

/* ------------------------------------------------------------------ */
/* Octree (pointer form): cubic cells (Sec. 3.1 quad/octree), children    */
/* in Morton order (x fastest, then y, then z)                           */
/* ------------------------------------------------------------------ */
struct ONode {
  int level;
  uint32_t i[3];
  std::unique_ptr<ONode> kid[8];
  int64_t leaf_index;
  bool is_leaf() const { return !kid[0]; }
  double h() const { return std::ldexp(1.0, -level); }
  double lo(int a) const { return i[a] * h(); }
  double hi(int a) const { return (i[a] + 1) * h(); }
};

void refine8(ONode* n) {
  for (int c = 0; c < 8; ++c) {
    n->kid[c].reset(new ONode());
    ONode* k = n->kid[c].get();
    k->level = n->level + 1;
    for (int a = 0; a < 3; ++a) k->i[a] = 2 * n->i[a] + ((c >> a) & 1);
    k->leaf_index = -1;
  }
}

void collect8(ONode* n, std::vector<ONode*>& out) {
  if (n->is_leaf()) { n->leaf_index = (int64_t)out.size(); out.push_back(n); return; }
  for (int c = 0; c < 8; ++c) collect8(n->kid[c].get(), out);
}

/* leaves whose closed box meets the closed box [lo, hi] */
void touching3(ONode* n, const double lo[3], const double hi[3], std::vector<ONode*>& out) {
  for (int a = 0; a < 3; ++a)
    if (n->lo(a) > hi[a] || lo[a] > n->hi(a)) return;
  if (n->is_leaf()) { out.push_back(n); return; }
  for (int c = 0; c < 8; ++c) touching3(n->kid[c].get(), lo, hi, out);
}

ONode* locate3(ONode* root, const double s[3]) {
  ONode* n = root;
  while (!n->is_leaf()) {
    const double hh = std::ldexp(1.0, -(n->level + 1));
    int c = 0;
    for (int a = 0; a < 3; ++a)
      if (s[a] >= (2 * n->i[a] + 1) * hh) c |= 1 << a;
    n = n->kid[c].get();
  }
  return n;
}

/* Morton code of three 10-bit coordinates (x in bits 0, 3, 6, ...) */
uint32_t morton10(uint32_t x, uint32_t y, uint32_t z) {
  uint32_t k = 0;
  for (int b = 0; b < 10; ++b) {
    k |= ((x >> b) & 1u) << (3 * b);
    k |= ((y >> b) & 1u) << (3 * b + 1);
    k |= ((z >> b) & 1u) << (3 * b + 2);
  }
  return k;
}

/* ------------------------------------------------------------------ */
/* Simulation state                                                    */
/* ------------------------------------------------------------------ */
struct SimBase {
  or_desc d;
  virtual ~SimBase() {}
};

template <class T> struct Particle {
  T s[3];
  T v[3];
  T b;            /* direct implicit: (dt/2) times the filtered acceleration, m/s */
  uint32_t w;
  uint32_t id;
  int64_t cell;   /* located leaf (2D) */
  bool alive;
};

template <class T> struct SpeciesK {
  /* host-derived constants, each computed in FP64 then rounded to T */
  double qm_dt, dt_L;
  uint32_t Tcand;
  double a_el, a_iz, v_iz2, mu2, vmax2, v_thg, a_cx, gmax;
  T qm_dtT, hqm_dtT, dt_LT, a_elT, a_izT, v_iz2T, mu2T, vmax2T, v_thgT, a_cxT, gmaxT;
};

template <class T> struct Sim : SimBase {
  static const int F = (sizeof(T) == 4) ? 24 : 32;   /* CIC fixed-point bits */
  std::vector<Particle<T>> p[2];
  SpeciesK<T> K[2];
  uint32_t next_id = 0;
  /* 1D */
  int N = 0;
  std::vector<T> En;            /* 1D: node E (momentum-conserving CIC) or cell E
                                   (energy-conserving CIC, N values + an unused one), in T */
  /* 2D */
  std::unique_ptr<QNode> root;
  std::vector<QNode*> leaves;
  std::vector<T> cornerE;       /* [leaf][corner][2] in T */
  std::vector<double> cornerE64;
  std::vector<double> cornerPhi; /* [leaf][corner]: potentials behind cornerE (if given) */
  std::vector<T> cellE;          /* [leaf][2]: cell-centred E (cloud-in-cell coupling), in T */
  std::vector<double> cellE64;
  /* 3D */
  std::unique_ptr<ONode> root3;
  std::vector<ONode*> leaves3;
  std::vector<T> cornerE3;       /* [leaf][corner][3] in T */
  std::vector<double> cornerE3_64;
  /* deposit */
  std::vector<uint64_t> Q[2];

  void derive() {
    for (int s = 0; s < d.nspecies; ++s) {
      const or_species& sp = d.species[s];
      SpeciesK<T>& k = K[s];
      k.qm_dt = (sp.charge * d.dt) / sp.mass;
      k.dt_L = d.dt / d.length;
      k.Tcand = 0; k.a_el = k.a_iz = k.v_iz2 = k.mu2 = k.vmax2 = k.v_thg = k.a_cx = k.gmax = 0.0;
      k.v_thg = std::sqrt((KB * d.gas_temperature) / d.gas_mass);
      if (sp.mcc == OR_MCC_ELECTRON) {
        double vmax = std::sqrt(((2.0 * QE) * sp.eps_max) / sp.mass);
        double sig_t = sp.sigma_el + sp.sigma_iz;
        double nu_max = (d.gas_density * sig_t) * vmax;
        double pnull = -std::expm1(-(nu_max * d.dt));
        k.Tcand = (uint32_t)std::floor(std::ldexp(pnull, 24));
        k.a_el = sp.sigma_el / (sig_t * vmax);
        k.a_iz = sp.sigma_iz / (sig_t * vmax);
        k.v_iz2 = ((2.0 * QE) * sp.eps_iz) / sp.mass;
        k.vmax2 = vmax * vmax;
        k.mu2 = (2.0 * sp.mass) / d.gas_mass;
      } else if (sp.mcc == OR_MCC_ION_CX) {
        double g = std::sqrt(((2.0 * QE) * sp.eps_max) / sp.mass) + 11.0 * k.v_thg;
        double nu_max = (d.gas_density * sp.sigma_cx) * g;
        double pnull = -std::expm1(-(nu_max * d.dt));
        k.Tcand = (uint32_t)std::floor(std::ldexp(pnull, 24));
        k.gmax = g;
        k.a_cx = 1.0 / g;
      }
      k.qm_dtT = (T)k.qm_dt;
      k.hqm_dtT = (T)0.5 * k.qm_dtT;
      k.dt_LT = (T)k.dt_L;
      k.a_elT = (T)k.a_el; k.a_izT = (T)k.a_iz; k.v_iz2T = (T)k.v_iz2; k.mu2T = (T)k.mu2;
      k.vmax2T = (T)k.vmax2; k.v_thgT = (T)k.v_thg; k.a_cxT = (T)k.a_cx; k.gmaxT = (T)k.gmax;
    }
  }

  int64_t nq() const {
    return d.dim == 1 ? (int64_t)N + 1 : d.dim == 3 ? (int64_t)leaves3.size() : (int64_t)leaves.size();
  }

  /* ---------------- 3D mesh: static octree ---------------- */
  /* base level everywhere, then every leaf whose closed box meets the
     closed ball (centre disk_cx, disk_cy, disk_cz, radius disk_r) refined
     until disk_level, then 2:1 balance across faces, edges and corners */
  bool build3() {
    if (d.min_level < 0 || d.max_level > 10 || d.min_level > d.max_level || d.base_level < d.min_level ||
        d.base_level > d.max_level)
      return false;
    if (d.nleaves > 0 || d.field_scheme != OR_FIELD_CIC_EM) return false;
    root3.reset(new ONode());
    root3->level = 0;
    root3->i[0] = root3->i[1] = root3->i[2] = 0;
    root3->leaf_index = -1;
    refine_uniform3(root3.get(), d.base_level);
    if (d.refine_disk) {
      const double c[3] = {d.disk_cx, d.disk_cy, d.disk_cz};
      bool changed = true;
      while (changed) {
        changed = false;
        std::vector<ONode*> lv;
        collect8(root3.get(), lv);
        for (ONode* n : lv) {
          if (n->level >= d.disk_level || n->level >= d.max_level) continue;
          double r2 = 0.0;
          for (int a = 0; a < 3; ++a) {
            const double g = std::max(std::max(n->lo(a) - c[a], 0.0), c[a] - n->hi(a));
            r2 = r2 + g * g;
          }
          if (r2 <= d.disk_r * d.disk_r) { refine8(n); changed = true; }
        }
      }
    }
    balance3();
    leaves3.clear();
    collect8(root3.get(), leaves3);
    cornerE3.assign(leaves3.size() * 24, (T)0);
    cornerE3_64.assign(leaves3.size() * 24, 0.0);
    for (int s = 0; s < 2; ++s) Q[s].assign(leaves3.size(), 0);
    return true;
  }

  void refine_uniform3(ONode* n, int L) {
    if (n->level >= L) return;
    refine8(n);
    for (int c = 0; c < 8; ++c) refine_uniform3(n->kid[c].get(), L);
  }

  int64_t balance3() {
    int64_t nref = 0;
    bool changed = true;
    while (changed) {
      changed = false;
      std::vector<ONode*> lv;
      collect8(root3.get(), lv);
      std::vector<ONode*> mark;
      for (ONode* a : lv) {
        const double lo[3] = {a->lo(0), a->lo(1), a->lo(2)}, hi[3] = {a->hi(0), a->hi(1), a->hi(2)};
        std::vector<ONode*> t;
        touching3(root3.get(), lo, hi, t);
        for (ONode* b : t)
          if (b->level > a->level + 1) { mark.push_back(a); break; }
      }
      for (ONode* a : mark) { refine8(a); ++nref; changed = true; }
    }
    return nref;
  }

  /* Nodal E on the octree from the potentials at each leaf's corners
     (corner c = a + 2b + 4e along x, y, z): each leaf's E = -grad of its
     trilinear potential at the corner -- x-component (f(0,b,e) - f(1,b,e))/h
     and likewise in y and z -- then at every node the mean over the leaves
     having the node as a corner (Sec. 3: nodal E), taken in octant order
     (the octant below the node in x first, then y, then z).  The leaf of an
     octant is the one holding the point half a finest cell from the node
     into it; the node is one of its corners when its coordinates are
     multiples of the leaf's size. */
  void corner_field3(const double* cphi) {
    const size_t nl = leaves3.size();
    std::vector<double> g(nl * 24);
    for (size_t l = 0; l < nl; ++l) {
      const double h = d.length * std::ldexp(1.0, -leaves3[l]->level);
      const double* f = &cphi[l * 8];
      for (int c = 0; c < 8; ++c) {
        const int a = c & 1, b = (c >> 1) & 1, e = c >> 2;
        g[l * 24 + c * 3 + 0] = (f[0 + 2 * b + 4 * e] - f[1 + 2 * b + 4 * e]) / h;
        g[l * 24 + c * 3 + 1] = (f[a + 0 + 4 * e] - f[a + 2 + 4 * e]) / h;
        g[l * 24 + c * 3 + 2] = (f[a + 2 * b + 0] - f[a + 2 * b + 4]) / h;
      }
    }
    for (size_t l = 0; l < nl; ++l) {
      const ONode* lf = leaves3[l];
      const uint32_t size = 1u << (10 - lf->level);
      for (int c = 0; c < 8; ++c) {
        uint32_t X[3];
        for (int a = 0; a < 3; ++a) X[a] = lf->i[a] * size + (((c >> a) & 1) ? size : 0u);
        double sum[3] = {0.0, 0.0, 0.0};
        int k = 0;
        for (int q = 0; q < 8; ++q) {
          bool inside = true;
          double pt[3];
          for (int a = 0; a < 3; ++a) {
            const int up = (q >> a) & 1;
            if ((up == 0 && X[a] == 0u) || (up == 1 && X[a] >= 1024u)) inside = false;
            pt[a] = ((double)X[a] + (up ? 0.5 : -0.5)) / 1024.0;
          }
          if (!inside) continue;
          const ONode* m = locate3(root3.get(), pt);
          const uint32_t ms = 1u << (10 - m->level);
          if (X[0] % ms || X[1] % ms || X[2] % ms) continue;   /* on an edge or face of m, not a corner */
          int mc = 0;
          for (int a = 0; a < 3; ++a)
            if (!((q >> a) & 1)) mc |= 1 << a;   /* m lies below the node along a: the node is its upper side */
          for (int a = 0; a < 3; ++a) sum[a] = sum[a] + g[(size_t)m->leaf_index * 24 + mc * 3 + a];
          ++k;
        }
        for (int a = 0; a < 3; ++a) {
          const double e = sum[a] / (double)k;
          cornerE3_64[l * 24 + c * 3 + a] = e;
          cornerE3[l * 24 + c * 3 + a] = (T)e;
        }
      }
    }
  }

  /* trilinear interpolation of the leaf's corner E at the particle (Sec. 3:
     gather from nodal E), weights ((x factor) (y factor)) (z factor),
     summed over the corners in order */
  void gather3d(const Particle<T>& q, T E[3]) const {
    const ONode* lf = leaves3[q.cell];
    const T sc = (T)std::ldexp(1.0, lf->level);
    T f[3];
    for (int a = 0; a < 3; ++a) f[a] = q.s[a] * sc - (T)lf->i[a];
    const T* ce = &cornerE3[q.cell * 24];
    for (int k = 0; k < 3; ++k) E[k] = (T)0;
    for (int c = 0; c < 8; ++c) {
      const T wx = (c & 1) ? f[0] : (T)1 - f[0];
      const T wy = ((c >> 1) & 1) ? f[1] : (T)1 - f[1];
      const T wz = (c >> 2) ? f[2] : (T)1 - f[2];
      const T w = (wx * wy) * wz;
      for (int k = 0; k < 3; ++k) E[k] = E[k] + w * ce[c * 3 + k];
    }
  }

  /* ---------------- mesh ---------------- */
  bool build() {
    derive();
    if (d.dim == 3) return build3();
    if (d.dim == 1) {
      N = d.ncells;
      if (N < 2) return false;
      En.assign(N + 1, (T)0);
    } else {
      if (d.min_level < 0 || d.max_level > 14 || d.min_level > d.max_level ||
          d.base_level < d.min_level || d.base_level > d.max_level) return false;
      root.reset(new QNode());
      root->level = 0; root->ix = root->iy = 0; root->parent = nullptr; root->leaf_index = -1;
      if (d.nleaves > 0) {
        if (!explicit_tree()) return false;
        relist();
        for (int s = 0; s < 2; ++s) Q[s].assign(nq(), 0);
        return true;
      }
      refine_uniform(root.get(), d.base_level);
      if (d.refine_disk) {
        bool changed = true;
        while (changed) {
          changed = false;
          std::vector<QNode*> lv;
          collect_leaves(root.get(), lv);
          for (QNode* n : lv) {
            if (n->level >= d.disk_level || n->level >= d.max_level) continue;
            double dx = std::max(std::max(n->x0() - d.disk_cx, 0.0), d.disk_cx - n->x1());
            double dy = std::max(std::max(n->y0() - d.disk_cy, 0.0), d.disk_cy - n->y1());
            if (dx * dx + dy * dy <= d.disk_r * d.disk_r) { refine_node(n); changed = true; }
          }
        }
      }
      balance();
      relist();
    }
    for (int s = 0; s < 2; ++s) Q[s].assign(nq(), 0);
    return true;
  }

  /* Tree given leaf by leaf (Morton order).  Each leaf is an aligned Morton
     range of 4^(16-level) keys; in Morton order they must follow each other
     without gap or overlap from key 0 to 2^32.  The pointer tree is grown by
     descending to each leaf.  An unbalanced tree is refused, not repaired. */
  bool explicit_tree() {
    if (!d.leaf_keys || !d.leaf_levels) return false;
    uint64_t pos = 0;
    for (int64_t i = 0; i < d.nleaves; ++i) {
      const int L = d.leaf_levels[i];
      if (L < d.min_level || L > d.max_level) return false;
      const uint64_t span = (uint64_t)1 << (2 * (16 - L));
      if ((uint64_t)d.leaf_keys[i] != pos) return false;
      pos += span;
      uint32_t X = 0, Y = 0;
      for (int b = 0; b < 16; ++b) {
        X |= ((d.leaf_keys[i] >> (2 * b)) & 1u) << b;
        Y |= ((d.leaf_keys[i] >> (2 * b + 1)) & 1u) << b;
      }
      const uint32_t ix = X >> (16 - L), iy = Y >> (16 - L);
      QNode* n = root.get();
      for (int l = 0; l < L; ++l) {
        if (n->is_leaf()) refine_node(n);
        const int c = (int)(((ix >> (L - 1 - l)) & 1u) + 2u * ((iy >> (L - 1 - l)) & 1u));
        n = n->kid[c].get();
      }
      if (!n->is_leaf()) return false;
    }
    if (pos != ((uint64_t)1 << 32)) return false;
    std::vector<QNode*> lv;
    collect_leaves(root.get(), lv);
    if ((int64_t)lv.size() != d.nleaves) return false;
    for (QNode* a : lv) {
      std::vector<QNode*> t;
      touching(root.get(), a->x0(), a->y0(), a->x1(), a->y1(), t);
      for (QNode* b : t)
        if (b->level > a->level + 1) return false;
    }
    return true;
  }

  void refine_uniform(QNode* n, int L) {
    if (n->level >= L) return;
    refine_node(n);
    for (int c = 0; c < 4; ++c) refine_uniform(n->kid[c].get(), L);
  }

  void relist() {
    leaves.clear();
    collect_leaves(root.get(), leaves);
    cornerE.assign(leaves.size() * 8, (T)0);
    cornerE64.assign(leaves.size() * 8, 0.0);
    cornerPhi.assign(leaves.size() * 4, 0.0);
    cellE.assign(leaves.size() * 2, (T)0);
    cellE64.assign(leaves.size() * 2, 0.0);
    for (int s = 0; s < 2; ++s) Q[s].assign(leaves.size(), 0);
  }

  /* 2:1 balance across faces and corners, by refinement only */
  int64_t balance() {
    int64_t nref = 0;
    bool changed = true;
    while (changed) {
      changed = false;
      std::vector<QNode*> lv;
      collect_leaves(root.get(), lv);
      std::vector<QNode*> mark;
      for (QNode* a : lv) {
        std::vector<QNode*> t;
        touching(root.get(), a->x0(), a->y0(), a->x1(), a->y1(), t);
        for (QNode* b : t)
          if (b->level > a->level + 1) { mark.push_back(a); break; }
      }
      for (QNode* a : mark) { refine_node(a); ++nref; changed = true; }
    }
    return nref;
  }

  int64_t locate_cell(const T s[3]) {
    if (d.dim == 1) return -1;
    if (d.dim == 3) {
      const double x[3] = {(double)s[0], (double)s[1], (double)s[2]};
      return locate3(root3.get(), x)->leaf_index;
    }
    return locate_node(root.get(), (double)s[0], (double)s[1])->leaf_index;
  }

  /* ---------------- particles ---------------- */
  int load(int sp, int64_t n, const double* s, const double* v, const uint32_t* w, const uint32_t* id) {
    if (sp < 0 || sp >= d.nspecies) return OR_E_ARG;
    std::vector<Particle<T>>& P = p[sp];
    P.clear();
    for (int64_t i = 0; i < n; ++i) {
      Particle<T> q;
      q.s[0] = (T)s[i * d.dim];
      q.s[1] = d.dim >= 2 ? (T)s[i * d.dim + 1] : (T)0;
      q.s[2] = d.dim == 3 ? (T)s[i * d.dim + 2] : (T)0;
      for (int c = 0; c < 3; ++c) q.v[c] = (T)v[i * 3 + c];
      q.w = w ? w[i] : 65536u;
      q.id = id ? id[i] : (uint32_t)i;
      q.b = (T)0;
      for (int c = 0; c < d.dim; ++c)
        if (!(q.s[c] >= (T)0 && q.s[c] < (T)1)) return OR_E_ARG;
      q.alive = true;
      q.cell = locate_cell(q.s);
      P.push_back(q);
      if (q.id + 1u > next_id) next_id = q.id + 1u;
    }
    std::sort(P.begin(), P.end(), [](const Particle<T>& a, const Particle<T>& b) { return a.id < b.id; });
    for (int o = 0; o < d.nspecies; ++o)
      for (const Particle<T>& q : p[o])
        if (q.id + 1u > next_id) next_id = q.id + 1u;
    return OR_OK;
  }

  /* ---------------- field gather ---------------- */
  /* E table from the node potentials ph[0..N]: node E by centred differences
     inside and second-order one-sided differences at the walls (momentum-
     conserving CIC), or cell E = (ph[i] - ph[i+1]) / dx for the N cells
     (energy-conserving CIC; e[N] unused, 0).  inv2dx = 1 / (2 dx). */
  void node_or_cell_e(const double* ph, double inv2dx, double* e) const {
    if (d.field_scheme == OR_FIELD_CIC_EC) {
      const double inv_dx = 2.0 * inv2dx;
      for (int i = 0; i < N; ++i) e[i] = (ph[i] - ph[i + 1]) * inv_dx;
      e[N] = 0.0;
      return;
    }
    e[0] = ((3.0 * ph[0] - 4.0 * ph[1]) + ph[2]) * inv2dx;
    for (int i = 1; i < N; ++i) e[i] = (ph[i - 1] - ph[i + 1]) * inv2dx;
    e[N] = ((-3.0 * ph[N] + 4.0 * ph[N - 1]) - ph[N - 2]) * inv2dx;
  }

  /* Momentum-conserving CIC: E interpolated linearly between the cell's two
     nodes (the same weights that assign its charge).  Energy-conserving CIC:
     the E of the particle's cell, the difference of its two node potentials
     (the derivative of the linear assignment function), Sec. 3. */
  T gather1d(T s) const {
    T g = s * (T)N;
    int64_t i = (int64_t)std::floor(g);
    if (i > N - 1) i = N - 1;
    if (d.field_scheme == OR_FIELD_CIC_EC) return En[i];
    T f = g - (T)i;
    return En[i] + f * (En[i + 1] - En[i]);
  }

  /* ---- cloud-in-cell on the quadtree (Sec. 3.1, Fig. 2) ----
     A particle in leaf l (level L, side h) is a square cloud of side h
     centred on it.  The cloud covers l and up to three level-L cells beside
     it: the direct neighbours on the particle's side of l's centre in x and
     in y, and the diagonal one; its bilinear area fractions, in fixed point
     with H = F/2 bits per axis, weight them.  Where the tree is not uniform
     those level-L cells are ghost cells (ghost cells at +-1 level in direct
     and diagonal neighbours, Sec. 3.1): one that lies inside a coarser leaf
     belongs to that leaf; one over finer leaves is shared among them in
     proportion to their area.  A ghost cell
     outside the domain is folded back across the wall onto the cell inside.
     The same fractions scatter the charge and gather the cell-centred field
     (the same shape function both ways, Sec. 3.1). */
  static const int H = F / 2;

  struct Cloud {
    uint32_t cx[4], cy[4];   /* centres of own, x-, y-, diagonal cell (16-bit units) */
    uint64_t share[4];       /* in units of 2^-F of the particle */
    T wt[4];                 /* the same fractions in T */
    int level;
  };

  Cloud cloud(const T s[2], int64_t cell) const {
    const QNode* lf = leaves[cell];
    const int L = lf->level;
    const uint32_t S = 1u << (16 - L);
    const T sc = (T)std::ldexp(1.0, L);
    const T gx = (s[0] * sc - (T)lf->ix) - (T)0.5, gy = (s[1] * sc - (T)lf->iy) - (T)0.5;
    const T ax = gx < (T)0 ? -gx : gx, ay = gy < (T)0 ? -gy : gy;
    const T one = (T)std::ldexp(1.0, H);
    const uint64_t rx = (uint64_t)std::rint(ax * one), ry = (uint64_t)std::rint(ay * one);
    const uint64_t o = (uint64_t)1 << H;
    Cloud c;
    c.level = L;
    const int64_t X = (int64_t)lf->ix * S + S / 2, Y = (int64_t)lf->iy * S + S / 2;
    const int64_t Xn = X + (gx >= (T)0 ? (int64_t)S : -(int64_t)S);
    const int64_t Yn = Y + (gy >= (T)0 ? (int64_t)S : -(int64_t)S);
    const bool xin = Xn >= 0 && Xn < 65536, yin = Yn >= 0 && Yn < 65536;
    const int64_t xs = xin ? Xn : X, ys = yin ? Yn : Y;   /* folded back at the walls */
    c.cx[0] = (uint32_t)X;  c.cy[0] = (uint32_t)Y;
    c.cx[1] = (uint32_t)xs; c.cy[1] = (uint32_t)Y;
    c.cx[2] = (uint32_t)X;  c.cy[2] = (uint32_t)ys;
    c.cx[3] = (uint32_t)xs; c.cy[3] = (uint32_t)ys;
    c.share[0] = (o - rx) * (o - ry);
    c.share[1] = rx * (o - ry);
    c.share[2] = (o - rx) * ry;
    c.share[3] = rx * ry;
    const T fx = (T)rx / one, fy = (T)ry / one;
    c.wt[0] = ((T)1 - fx) * ((T)1 - fy);
    c.wt[1] = fx * ((T)1 - fy);
    c.wt[2] = ((T)1 - fx) * fy;
    c.wt[3] = fx * fy;
    return c;
  }

  /* The leaves that make up the level-L cell centred at (X, Y) (16-bit
     units): the one leaf holding it (at level L or coarser), or the finer
     leaves tiling it, which follow each other in Morton order.  Returns the
     index of the first and the count; level differences in 'dl'. */
  int64_t cell_leaves(uint32_t X, uint32_t Y, int L, std::vector<int>& dl) const {
    const uint32_t S = 1u << (16 - L);
    const uint32_t X0 = X - S / 2, Y0 = Y - S / 2;
    const QNode* n = locate_node(root.get(), X0 / 65536.0, Y0 / 65536.0);
    dl.clear();
    if (n->level <= L) {
      dl.push_back(0);
      return n->leaf_index;
    }
    const double x0 = X0 / 65536.0, y0 = Y0 / 65536.0, x1 = (X0 + S) / 65536.0, y1 = (Y0 + S) / 65536.0;
    for (size_t l = (size_t)n->leaf_index; l < leaves.size(); ++l) {
      const QNode* m = leaves[l];
      if (!(m->x0() >= x0 && m->x1() <= x1 && m->y0() >= y0 && m->y1() <= y1)) break;
      dl.push_back(m->level - L);
    }
    return n->leaf_index;
  }

  /* units of charge into the level-L cell centred at (X, Y): all to the leaf
     holding it, or to the finer leaves tiling it in proportion to their area
     (units / 4^(level difference), rounded down; what the rounding leaves
     goes to the first of them) */
  void scatter_cell(uint32_t X, uint32_t Y, int L, uint64_t units, std::vector<uint64_t>& Qs) const {
    std::vector<int> dl;
    const int64_t first = cell_leaves(X, Y, L, dl);
    uint64_t given = 0;
    for (size_t k = 0; k < dl.size(); ++k) {
      const uint64_t part = units >> (2 * dl[k]);
      Qs[first + (int64_t)k] += part;
      given += part;
    }
    Qs[first] += units - given;
  }

  /* cell-centred field of the level-L cell centred at (X, Y): its leaf's, or
     the area-weighted mean of the finer leaves tiling it, summed in Morton
     order */
  void gather_cell(uint32_t X, uint32_t Y, int L, T E[2]) const {
    std::vector<int> dl;
    const int64_t first = cell_leaves(X, Y, L, dl);
    E[0] = E[1] = (T)0;
    for (size_t k = 0; k < dl.size(); ++k) {
      const T f = (T)std::ldexp(1.0, -2 * dl[k]);
      for (int c = 0; c < 2; ++c) E[c] = E[c] + cellE[(first + (int64_t)k) * 2 + c] * f;
    }
  }

  void gather_cic_amr(const T s[2], int64_t cell, T E[2]) const {
    const Cloud c = cloud(s, cell);
    T e[4][2];
    for (int k = 0; k < 4; ++k) gather_cell(c.cx[k], c.cy[k], c.level, e[k]);
    for (int m = 0; m < 2; ++m)
      E[m] = ((c.wt[0] * e[0][m] + c.wt[1] * e[1][m]) + c.wt[2] * e[2][m]) + c.wt[3] * e[3][m];
  }

  void gather2d(const Particle<T>& q, T E[2]) const {
    if (d.field_scheme == OR_FIELD_CIC_AMR) {
      gather_cic_amr(q.s, q.cell, E);
      return;
    }
    const QNode* lf = leaves[q.cell];
    T sc = (T)std::ldexp(1.0, lf->level);
    T xi = q.s[0] * sc - (T)lf->ix;
    T eta = q.s[1] * sc - (T)lf->iy;
    T w00 = ((T)1 - xi) * ((T)1 - eta);
    T w10 = xi * ((T)1 - eta);
    T w01 = ((T)1 - xi) * eta;
    T w11 = xi * eta;
    const T* c = &cornerE[q.cell * 8];
    for (int k = 0; k < 2; ++k)
      E[k] = ((w00 * c[0 + k] + w10 * c[2 + k]) + w01 * c[4 + k]) + w11 * c[6 + k];
  }

  /* wall rule on one coordinate: true if the particle stays */
  bool wall(T& s, T& v, bool& lost_reflect) const {
    if (s >= (T)0 && s < (T)1) return true;
    if (d.particle_bc == OR_ABSORB) return false;
    if (s < (T)0) {
      s = -s;
      v = -v;
    } else if (s >= (T)1) {
      s = (T)2 - s;
      v = -v;
      if (s == (T)1) s = std::nextafter((T)1, (T)0);
    }
    if (s >= (T)0 && s < (T)1) return true;
    lost_reflect = true;
    return false;
  }

  /* ---------------- MCC (null collision) ---------------- */
  struct Birth { uint32_t parent; T s[3]; int64_t cell; T ve[3]; T vi[3]; uint32_t w; };

  void mcc(int sp, Particle<T>& q, uint32_t step, std::vector<Birth>& births, or_stats* st) {
    const SpeciesK<T>& k = K[sp];
    const or_species& sd = d.species[sp];
    Stream rs(d.seed, d.instance_key, q.id, step);
    uint32_t r0 = rs.next();
    uint32_t r1 = rs.next();
    if ((r0 >> 8) >= k.Tcand) return;
    T u1 = uniform<T>(r1);
    T* v = q.v;
    if (sd.mcc == OR_MCC_ELECTRON) {
      T v2 = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
      if (v2 > k.vmax2T) st->numax_violations[sp]++;
      T vmag = std::sqrt(v2);
      T x_el = k.a_elT * vmag;
      if (u1 < x_el) {
        T dd[3];
        iso_dir<T>(rs, dd);
        T vd = (v[0] * dd[0] + v[1] * dd[1]) + v[2] * dd[2];
        T vp2 = v2 - k.mu2T * (v2 - vmag * vd);
        if (vp2 < (T)0) vp2 = (T)0;
        T vpm = std::sqrt(vp2);
        for (int c = 0; c < 3; ++c) v[c] = vpm * dd[c];
        st->elastic++;
      } else if (v2 >= k.v_iz2T && u1 < x_el + k.a_izT * vmag) {
        T u0 = uniform<T>(rs.next());
        T v2ex = v2 - k.v_iz2T;
        T v2a = u0 * v2ex;
        T v2b = v2ex - v2a;
        T d1[3], d2[3];
        iso_dir<T>(rs, d1);
        iso_dir<T>(rs, d2);
        T va = std::sqrt(v2a), vb = std::sqrt(v2b);
        Birth b;
        b.parent = q.id;
        b.s[0] = q.s[0]; b.s[1] = q.s[1]; b.s[2] = q.s[2]; b.cell = q.cell; b.w = q.w;
        for (int c = 0; c < 3; ++c) { v[c] = va * d1[c]; b.ve[c] = vb * d2[c]; }
        for (int c = 0; c < 3; ++c) b.vi[c] = k.v_thgT * gauss12<T>(rs);
        births.push_back(b);
        st->ionization++;
      }
    } else if (sd.mcc == OR_MCC_ION_CX) {
      T vn[3];
      for (int c = 0; c < 3; ++c) vn[c] = k.v_thgT * gauss12<T>(rs);
      T dx = v[0] - vn[0], dy = v[1] - vn[1], dz = v[2] - vn[2];
      T g = std::sqrt((dx * dx + dy * dy) + dz * dz);
      if (g > k.gmaxT) st->numax_violations[sp]++;
      if (u1 < k.a_cxT * g) {
        for (int c = 0; c < 3; ++c) v[c] = vn[c];
        st->cx++;
      }
    }
  }

  /* ---------------- deposit ---------------- */
  void deposit() {
    for (int s = 0; s < 2; ++s) std::fill(Q[s].begin(), Q[s].end(), 0);
    const uint64_t one = (uint64_t)1 << F;
    for (int sp = 0; sp < d.nspecies; ++sp) {
      for (const Particle<T>& q : p[sp]) {
        if (!q.alive) continue;
        if (d.dim == 1) {
          T g = q.s[0] * (T)N;
          int64_t i = (int64_t)std::floor(g);
          if (i > N - 1) i = N - 1;
          T f = g - (T)i;
          uint64_t r = (uint64_t)(int64_t)std::rint(f * (T)std::ldexp(1.0, F));
          Q[sp][i] += (uint64_t)q.w * (one - r);
          Q[sp][i + 1] += (uint64_t)q.w * r;
        } else if (d.field_scheme == OR_FIELD_CIC_AMR) {
          const Cloud c = cloud(q.s, q.cell);
          for (int k = 0; k < 4; ++k)
            if (c.share[k]) scatter_cell(c.cx[k], c.cy[k], c.level, (uint64_t)q.w * c.share[k], Q[sp]);
        } else {
          Q[sp][q.cell] += (uint64_t)q.w;
        }
      }
    }
  }

  /* ---------------- one step of the particle loop ---------------- */
  int step(uint32_t n, or_stats* st) {
    std::vector<Birth> births;
    for (int sp = 0; sp < d.nspecies; ++sp) {
      const SpeciesK<T>& k = K[sp];
      for (Particle<T>& q : p[sp]) {
        if (!q.alive) continue;
        st->alive_start[sp]++;
        bool lost_r = false;
        if (d.dim == 1) {
          T E = gather1d(q.s[0]);
          q.v[0] = q.v[0] + k.qm_dtT * E;
          q.s[0] = q.s[0] + q.v[0] * k.dt_LT;
          if (!wall(q.s[0], q.v[0], lost_r)) {
            q.alive = false;
            st->absorbed[sp]++;
            if (lost_r) st->lost_reflect++;
            continue;
          }
        } else if (d.dim == 3) {
          T E[3];
          gather3d(q, E);
          for (int a = 0; a < 3; ++a) q.v[a] = q.v[a] + k.qm_dtT * E[a];
          for (int a = 0; a < 3; ++a) q.s[a] = q.s[a] + q.v[a] * k.dt_LT;
          bool ok = true;
          for (int a = 0; a < 3 && ok; ++a) ok = wall(q.s[a], q.v[a], lost_r);
          if (!ok) {
            q.alive = false;
            st->absorbed[sp]++;
            if (lost_r) st->lost_reflect++;
            continue;
          }
          q.cell = locate_cell(q.s);
        } else {
          T E[2];
          gather2d(q, E);
          q.v[0] = q.v[0] + k.qm_dtT * E[0];
          q.v[1] = q.v[1] + k.qm_dtT * E[1];
          q.s[0] = q.s[0] + q.v[0] * k.dt_LT;
          q.s[1] = q.s[1] + q.v[1] * k.dt_LT;
          bool okx = wall(q.s[0], q.v[0], lost_r);
          bool oky = okx && wall(q.s[1], q.v[1], lost_r);
          if (!(okx && oky)) {
            q.alive = false;
            st->absorbed[sp]++;
            if (lost_r) st->lost_reflect++;
            continue;
          }
          q.cell = locate_cell(q.s);
        }
        if (d.species[sp].mcc != OR_MCC_NONE) mcc(sp, q, n, births, st);
      }
    }
    return finish_step(births, st);
  }

  /* births appended, the absorbed removed, the deposit of the step */
  int finish_step(std::vector<Birth>& births, or_stats* st) {
    /* births: sorted by parent id; rank r -> electron next_id+2r, ion +2r+1 */
    std::sort(births.begin(), births.end(), [](const Birth& a, const Birth& b) { return a.parent < b.parent; });
    if (!births.empty()) {
      if (d.nspecies < 2) return OR_E_STATE;
      uint64_t need = (uint64_t)next_id + 2ull * births.size();
      if (need > 0xFFFFFFFFull) return OR_E_CAPACITY;
      for (size_t r = 0; r < births.size(); ++r) {
        const Birth& b = births[r];
        Particle<T> e, i;
        e.s[0] = i.s[0] = b.s[0];
        e.s[1] = i.s[1] = b.s[1];
        e.s[2] = i.s[2] = b.s[2];
        e.cell = i.cell = b.cell;
        e.w = i.w = b.w;
        e.b = i.b = (T)0;
        e.alive = i.alive = true;
        for (int c = 0; c < 3; ++c) { e.v[c] = b.ve[c]; i.v[c] = b.vi[c]; }
        e.id = next_id + 2u * (uint32_t)r;
        i.id = e.id + 1u;
        p[0].push_back(e);
        p[1].push_back(i);
      }
      next_id += 2u * (uint32_t)births.size();
      st->births += (int64_t)births.size();
    }
    /* remove the absorbed, keeping id order */
    for (int sp = 0; sp < d.nspecies; ++sp)
      p[sp].erase(std::remove_if(p[sp].begin(), p[sp].end(), [](const Particle<T>& q) { return !q.alive; }),
                  p[sp].end());
    deposit();
    return OR_OK;
  }

  /* ---------------- 1D direct implicit step (Sec. 3: DIPIC) ----------------
     The D1 scheme of direct implicit PIC, with the particle velocity v at
     half steps and b = (dt/2) abar, abar the filtered acceleration:
       predictor   v~ = v + b,   x~ = x + dt v~                (walls apply)
       field       -d/dx[(1 + chi) dphi/dx] = rho~ / eps0 at t_{n+1}, rho~
                   and chi from the charge at the predicted positions,
                   chi = sum_s (q_s / m_s) (dt^2 / 2) rho~_s / eps0
       corrector   a = (q/m) E_{n+1}(x~),  v = v~ + (dt/2) a,
                   x = x~ + dt (dt/2) a,   b = (b + (dt/2) a) / 2  (walls apply)
     then collisions and births (a newborn has b = 0) and the deposit.
     Readings: chi at the nodes from the CIC charge sums of each species
     over the node's cell (a wall node's half cell: twice its sum over dx,
     the density there; over a whole cell the wall face of a uniform
     plasma would see a quarter less susceptibility than the interior, and
     at large w_p dt the sheets beside the walls grow); the face
     coefficient 1 + (chi_i + chi_{i+1}) / 2; the variable-coefficient
     system solved by the Thomas algorithm in FP64 (forward elimination
     from node 1, back substitution from node N-1). */
  double chi_coef(int sp) const {
    const or_species& s = d.species[sp];
    const double dx = d.length / N;
    return (((s.charge / s.mass) * ((d.dt * d.dt) * 0.5)) * (((s.charge * s.w0) * std::ldexp(1.0, -(16 + F))) / dx)) /
           EPS0;
  }

  void solve1d_implicit(double phi_left, double* phi_out = nullptr, double* chi_out = nullptr) {
    std::vector<double> chi(N + 1, 0.0), f(N), ph(N + 1, 0.0);
    for (int i = 0; i <= N; ++i) {
      double c = 0.0;
      for (int sp = 0; sp < d.nspecies; ++sp) c = c + chi_coef(sp) * (double)(int64_t)Q[sp][i];
      chi[i] = (i == 0 || i == N) ? 2.0 * c : c;   /* a wall node's charge fills half a cell */
    }
    for (int i = 0; i < N; ++i) f[i] = 1.0 + (chi[i] + chi[i + 1]) * 0.5;   /* face i + 1/2 */
    /* interior nodes 1 .. N-1: -f[i-1] ph[i-1] + (f[i-1] + f[i]) ph[i] - f[i] ph[i+1] = rhs[i] */
    std::vector<double> cp(N, 0.0), dp(N, 0.0);
    for (int i = 1; i < N; ++i) {
      double r = 0.0;
      for (int sp = 0; sp < d.nspecies; ++sp) r = r + (double)(int64_t)Q[sp][i] * kappa(sp);
      if (i == 1) r = r + f[0] * phi_left;
      const double a = -f[i - 1], bb = f[i - 1] + f[i], c = -f[i];
      if (i == 1) {
        cp[i] = c / bb;
        dp[i] = r / bb;
      } else {
        const double m = bb - a * cp[i - 1];
        cp[i] = c / m;
        dp[i] = (r - a * dp[i - 1]) / m;
      }
    }
    ph[0] = phi_left;
    ph[N] = 0.0;
    ph[N - 1] = dp[N - 1];
    for (int i = N - 2; i >= 1; --i) ph[i] = dp[i] - cp[i] * ph[i + 1];
    const double inv2dx = 1.0 / (2.0 * (d.length / N));
    std::vector<double> e(N + 1);
    node_or_cell_e(ph.data(), inv2dx, e.data());
    for (int i = 0; i <= N; ++i) {
      En[i] = (T)e[i];
      if (phi_out) phi_out[i] = ph[i];
      if (chi_out) chi_out[i] = chi[i];
    }
  }

  int step_dipic(uint32_t n, double phi_left, or_stats* st) {
    std::vector<Birth> births;
    for (int sp = 0; sp < d.nspecies; ++sp) {
      const SpeciesK<T>& k = K[sp];
      for (Particle<T>& q : p[sp]) {
        if (!q.alive) continue;
        st->alive_start[sp]++;
        q.v[0] = q.v[0] + q.b;
        q.s[0] = q.s[0] + q.v[0] * k.dt_LT;
        bool lost_r = false;
        if (!wall(q.s[0], q.v[0], lost_r)) {
          q.alive = false;
          st->absorbed[sp]++;
          if (lost_r) st->lost_reflect++;
        }
      }
    }
    deposit();                    /* charge at the predicted positions */
    solve1d_implicit(phi_left);   /* E at t_{n+1} */
    for (int sp = 0; sp < d.nspecies; ++sp) {
      const SpeciesK<T>& k = K[sp];
      for (Particle<T>& q : p[sp]) {
        if (!q.alive) continue;
        const T dv = k.hqm_dtT * gather1d(q.s[0]);
        q.v[0] = q.v[0] + dv;
        q.s[0] = q.s[0] + dv * k.dt_LT;
        q.b = (q.b + dv) * (T)0.5;
        bool lost_r = false;
        if (!wall(q.s[0], q.v[0], lost_r)) {
          q.alive = false;
          st->absorbed[sp]++;
          if (lost_r) st->lost_reflect++;
          continue;
        }
        if (d.species[sp].mcc != OR_MCC_NONE) mcc(sp, q, n, births, st);
      }
    }
    return finish_step(births, st);
  }

  /* ---------------- 1D Poisson (Thomas) ---------------- */
  double kappa(int sp) const {
    const or_species& s = d.species[sp];
    if (d.dim == 1) {
      double dx = d.length / N;
      return (((s.charge * s.w0) * std::ldexp(1.0, -(16 + F))) * dx) / EPS0;
    }
    const int f2 = d.field_scheme == OR_FIELD_CIC_AMR ? F : 0;   /* cloud shares carry F more bits */
    return (((s.charge * s.w0) * std::ldexp(1.0, -(16 + f2))) / d.depth_z) / EPS0;
  }

  /* charge density of the latest deposit: the integer sums scaled to
     coulombs (w_units = 2^16 carries w0 real particles; 1D shares carry F
     more bits) over the cell volume per unit area (dx, 1D) or per leaf area
     and depth (h^2 depth_z, 2D); no per-level weighting (Sec. 3.1) */
  void rho(double* out) const {
    for (int64_t i = 0; i < nq(); ++i) {
      double r = 0.0;
      for (int sp = 0; sp < d.nspecies; ++sp) {
        const or_species& s = d.species[sp];
        const double units = (double)(int64_t)Q[sp][i];
        if (d.dim == 1)
          r = r + ((units * std::ldexp(1.0, -(16 + F))) * (s.charge * s.w0)) / (d.length / N);
        else if (d.dim == 3) {
          const double h = d.length * std::ldexp(1.0, -leaves3[i]->level);
          r = r + ((units * std::ldexp(1.0, -16)) * (s.charge * s.w0)) / ((h * h) * h);
        } else {
          const double h = d.length * std::ldexp(1.0, -leaves[i]->level);
          const int f2 = d.field_scheme == OR_FIELD_CIC_AMR ? F : 0;
          r = r + ((units * std::ldexp(1.0, -(16 + f2))) * (s.charge * s.w0)) / ((h * h) * d.depth_z);
        }
      }
      out[i] = r;
    }
  }

  double rhs_cell(int64_t i) const {
    double b = 0.0;
    for (int sp = 0; sp < d.nspecies; ++sp) b = b + (double)(int64_t)Q[sp][i] * kappa(sp);
    return b;
  }

  /* 1D Poisson on the nodes (Sec. 3; potential phi_0 = V(t) on the powered
     wall, phi_N = 0 on the grounded one):
       2 phi_i - phi_{i-1} - phi_{i+1} = c_i,   c_i = sum_s kappa_s Q_s,i,
     for i = 1 .. N-1.  Its exact solution, from the inverse of
     tridiag(-1, 2, -1), (A^-1)_ij = min(i, j) (N - max(i, j)) / N, is
       phi_i = V (N - i) / N
             + sum_s (kappa_s / N) [ (N - i) sum_{j <= i} j Q_s,j
                                     + i sum_{j > i} (N - j) Q_s,j ].
     The Q are integer charge sums, so each bracket is an exact integer
     (formed here in 128-bit arithmetic with running sums) and is rounded to
     double once; the rest is a fixed short sequence of double operations.
     The charge at the wall nodes does not enter (Dirichlet nodes). */
  void solve1d(double phi_left, double* phi, double* E) {
    typedef unsigned __int128 u128;
    std::vector<double> ph(N + 1, 0.0);
    ph[0] = phi_left;
    ph[N] = 0.0;
    std::vector<u128> P1[2], P2[2];
    u128 T2[2] = {0, 0};
    for (int sp = 0; sp < d.nspecies; ++sp) {
      P1[sp].assign(N, 0);
      P2[sp].assign(N, 0);
      u128 a = 0, b = 0;
      for (int j = 1; j < N; ++j) {
        a += (u128)(uint64_t)j * (u128)Q[sp][j];
        b += (u128)(uint64_t)(N - j) * (u128)Q[sp][j];
        P1[sp][j] = a;
        P2[sp][j] = b;
      }
      T2[sp] = b;
    }
    for (int i = 1; i < N; ++i) {
      double v = (phi_left * (double)(N - i)) / (double)N;
      for (int sp = 0; sp < d.nspecies; ++sp) {
        const u128 D = (u128)(uint64_t)(N - i) * P1[sp][i] + (u128)(uint64_t)i * (T2[sp] - P2[sp][i]);
        v = v + ((double)D * kappa(sp)) / (double)N;
      }
      ph[i] = v;
    }
    double inv2dx = 1.0 / (2.0 * (d.length / N));
    std::vector<double> e(N + 1);
    node_or_cell_e(ph.data(), inv2dx, e.data());
    for (int i = 0; i <= N; ++i) {
      En[i] = (T)e[i];
      if (phi) phi[i] = ph[i];
      if (E) E[i] = e[i];
    }
  }

  /* ---------------- 2D field: nodes, corner gradients, nodal E -------- */
  struct NodeRef { int q; int64_t leaf; int corner; };
  typedef std::map<std::pair<uint32_t, uint32_t>, std::vector<NodeRef>> NodeMap;

  void node_map(NodeMap& m) const {
    for (size_t l = 0; l < leaves.size(); ++l) {
      const QNode* lf = leaves[l];
      uint32_t sh = 16 - lf->level;
      for (int c = 0; c < 4; ++c) {
        int a = c & 1, b = c >> 1;
        uint32_t X = (lf->ix + a) << sh, Y = (lf->iy + b) << sh;
        int quad = (1 - a) + 2 * (1 - b);   /* SW=0, SE=1, NW=2, NE=3 relative to the node */
        m[{X, Y}].push_back(NodeRef{quad, (int64_t)l, c});
      }
    }
    for (auto& kv : m)
      std::sort(kv.second.begin(), kv.second.end(), [](const NodeRef& x, const NodeRef& y) { return x.q < y.q; });
  }

  bool dirichlet_node(uint32_t X, uint32_t Y, double& val) const {
    const uint32_t E = 65536u;
    if (X == 0 && d.field_bc[0] == OR_WALL_DIRICHLET) { val = d.wall_phi[0]; return true; }
    if (X == E && d.field_bc[1] == OR_WALL_DIRICHLET) { val = d.wall_phi[1]; return true; }
    if (Y == 0 && d.field_bc[2] == OR_WALL_DIRICHLET) { val = d.wall_phi[2]; return true; }
    if (Y == E && d.field_bc[3] == OR_WALL_DIRICHLET) { val = d.wall_phi[3]; return true; }
    return false;
  }

  /* corner potentials per leaf -> corner gradients -> nodal E table */
  void corner_field_from_corner_phi(const std::vector<double>& cphi) {
    size_t nl = leaves.size();
    cornerPhi = cphi;
    std::vector<double> g(nl * 8);
    for (size_t l = 0; l < nl; ++l) {
      double h = d.length * std::ldexp(1.0, -leaves[l]->level);
      const double* f = &cphi[l * 4];   /* corners (a,b): 0=(0,0) 1=(1,0) 2=(0,1) 3=(1,1) */
      for (int c = 0; c < 4; ++c) {
        int a = c & 1, b = c >> 1;
        g[l * 8 + c * 2 + 0] = (f[0 + 2 * b] - f[1 + 2 * b]) / h;
        g[l * 8 + c * 2 + 1] = (f[a + 0] - f[a + 2]) / h;
      }
    }
    NodeMap m;
    node_map(m);
    for (auto& kv : m) {
      const std::vector<NodeRef>& refs = kv.second;
      double sx = 0.0, sy = 0.0;
      for (const NodeRef& r : refs) {
        sx = sx + g[r.leaf * 8 + r.corner * 2 + 0];
        sy = sy + g[r.leaf * 8 + r.corner * 2 + 1];
      }
      double k = (double)refs.size();
      double ex = sx / k, ey = sy / k;
      for (const NodeRef& r : refs) {
        cornerE64[r.leaf * 8 + r.corner * 2 + 0] = ex;
        cornerE64[r.leaf * 8 + r.corner * 2 + 1] = ey;
      }
    }
    for (size_t i = 0; i < cornerE64.size(); ++i) cornerE[i] = (T)cornerE64[i];
    cell_e_from_corners();
  }

  /* cell-centred E of each leaf: the mean of its four nodal E values (the
     gradient of its bilinear potential at the centre when the nodal E come
     from that potential) */
  void cell_e_from_corners() {
    for (size_t l = 0; l < leaves.size(); ++l)
      for (int k = 0; k < 2; ++k) {
        const double* c = &cornerE64[l * 8];
        cellE64[l * 2 + k] = 0.25 * ((c[0 + k] + c[2 + k]) + (c[4 + k] + c[6 + k]));
        cellE[l * 2 + k] = (T)cellE64[l * 2 + k];
      }
  }

  void corner_field_from_cell_phi(const double* phi) {
    size_t nl = leaves.size();
    std::vector<double> cphi(nl * 4);
    NodeMap m;
    node_map(m);
    for (auto& kv : m) {
      double val;
      if (!dirichlet_node(kv.first.first, kv.first.second, val)) {
        double s = 0.0;
        for (const NodeRef& r : kv.second) s = s + phi[r.leaf];
        val = s / (double)kv.second.size();
      }
      for (const NodeRef& r : kv.second) cphi[r.leaf * 4 + r.corner] = val;
    }
    corner_field_from_corner_phi(cphi);
  }

  /* ---------------- 2D cell-centred FV operator ---------------- */
  struct Row { std::vector<std::pair<int64_t, double>> off; double diag; double bnd; };

  void assemble(std::vector<Row>& rows) const {
    size_t nl = leaves.size();
    rows.assign(nl, Row());
    for (size_t l = 0; l < nl; ++l) {
      QNode* a = leaves[l];
      Row& R = rows[l];
      R.diag = 0.0; R.bnd = 0.0;
      std::vector<QNode*> t;
      touching(root.get(), a->x0(), a->y0(), a->x1(), a->y1(), t);
      for (QNode* b : t) {
        if (b == a) continue;
        double ov;
        bool face = false;
        if (b->x0() == a->x1() || b->x1() == a->x0()) {
          ov = std::min(a->y1(), b->y1()) - std::max(a->y0(), b->y0());
          face = ov > 0.0;
        }
        if (!face && (b->y0() == a->y1() || b->y1() == a->y0())) {
          ov = std::min(a->x1(), b->x1()) - std::max(a->x0(), b->x0());
          face = ov > 0.0;
        }
        if (!face) continue;
        double ha = a->h(), hb = b->h();
        double c = std::min(ha, hb) / ((ha + hb) / 2.0);
        R.off.push_back({b->leaf_index, c});
        R.diag = R.diag + c;
      }
      const int side_on[4] = {a->x0() == 0.0, a->x1() == 1.0, a->y0() == 0.0, a->y1() == 1.0};
      for (int w = 0; w < 4; ++w)
        if (side_on[w] && d.field_bc[w] == OR_WALL_DIRICHLET) {
          R.diag = R.diag + 2.0;
          R.bnd = R.bnd + 2.0 * d.wall_phi[w];
        }
    }
  }

  int cg2d(const double* init, double rtol, int maxit, double* out, int* iters, double* relres) {
    std::vector<Row> rows;
    assemble(rows);
    size_t n = rows.size();
    std::vector<double> b(n), x(n, 0.0), r(n), z(n), pp(n), q(n);
    for (size_t i = 0; i < n; ++i) b[i] = rhs_cell(i) + rows[i].bnd;
    if (init) for (size_t i = 0; i < n; ++i) x[i] = init[i];
    auto apply = [&](const std::vector<double>& xx, std::vector<double>& yy) {
      for (size_t i = 0; i < n; ++i) {
        double y = rows[i].diag * xx[i];
        for (auto& e : rows[i].off) y = y - e.second * xx[e.first];
        yy[i] = y;
      }
    };
    auto dot = [&](const std::vector<double>& u, const std::vector<double>& w) {
      double s = 0.0;
      for (size_t i = 0; i < n; ++i) s = s + u[i] * w[i];
      return s;
    };
    apply(x, q);
    for (size_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    for (size_t i = 0; i < n; ++i) z[i] = r[i] / rows[i].diag;
    pp = z;
    double rz = dot(r, z);
    double bn = std::sqrt(dot(b, b));
    int it = 0;
    double rn = std::sqrt(dot(r, r));
    while (it < maxit && rn > rtol * bn) {
      apply(pp, q);
      double alpha = rz / dot(pp, q);
      for (size_t i = 0; i < n; ++i) { x[i] = x[i] + alpha * pp[i]; r[i] = r[i] - alpha * q[i]; }
      for (size_t i = 0; i < n; ++i) z[i] = r[i] / rows[i].diag;
      double rzn = dot(r, z);
      double beta = rzn / rz;
      rz = rzn;
      for (size_t i = 0; i < n; ++i) pp[i] = z[i] + beta * pp[i];
      rn = std::sqrt(dot(r, r));
      ++it;
    }
    for (size_t i = 0; i < n; ++i) out[i] = x[i];
    *iters = it;
    *relres = bn > 0 ? rn / bn : 0.0;
    corner_field_from_cell_phi(out);
    return (rn <= rtol * bn) ? OR_OK : OR_E_STATE;
  }

  /* ---------------- adapt: counts, coarsen, refine, balance, split/merge */
  void relocate_all() {
    for (int sp = 0; sp < d.nspecies; ++sp)
      for (Particle<T>& q : p[sp]) q.cell = locate_cell(q.s);
  }

  std::vector<int64_t> counts(int sp) const {
    std::vector<int64_t> c(leaves.size(), 0);
    for (const Particle<T>& q : p[sp]) c[q.cell]++;
    return c;
  }

  int64_t nmax(const std::vector<std::vector<int64_t>>& c, int64_t l) const {
    int64_t m = 0;
    for (int sp = 0; sp < d.nspecies; ++sp) m = std::max(m, c[sp][l]);
    return m;
  }

  int adapt(int n_lo, int n_hi, or_adapt_stats* st) {
    std::memset(st, 0, sizeof(*st));
    relocate_all();
    std::vector<std::vector<int64_t>> c(d.nspecies);
    for (int sp = 0; sp < d.nspecies; ++sp) c[sp] = counts(sp);
    /* decisions on the pre-pass tree */
    std::vector<QNode*> coarsen, refine;
    for (size_t l = 0; l < leaves.size(); ++l) {
      QNode* a = leaves[l];
      if (nmax(c, l) > n_hi && a->level < d.max_level) refine.push_back(a);
      QNode* P = a->parent;
      if (!P || a != P->kid[0].get() || a->level <= d.min_level) continue;
      bool all_leaves = true;
      for (int k = 0; k < 4; ++k) all_leaves = all_leaves && P->kid[k]->is_leaf();
      if (!all_leaves) continue;
      int64_t smax = 0, cmin = INT64_MAX;
      for (int sp = 0; sp < d.nspecies; ++sp) {
        int64_t s = 0;
        for (int k = 0; k < 4; ++k) s += c[sp][P->kid[k]->leaf_index];
        smax = std::max(smax, s);
      }
      for (int k = 0; k < 4; ++k) cmin = std::min(cmin, nmax(c, P->kid[k]->leaf_index));
      if (!(smax <= n_hi && cmin < n_lo)) continue;
      std::vector<QNode*> t;
      touching(root.get(), P->x0(), P->y0(), P->x1(), P->y1(), t);
      bool ok = true;
      for (QNode* b : t) {
        bool inside = b->x0() >= P->x0() && b->x1() <= P->x1() && b->y0() >= P->y0() && b->y1() <= P->y1();
        if (!inside && b->level > P->level + 1) { ok = false; break; }
      }
      if (ok) coarsen.push_back(P);
    }
    for (QNode* P : coarsen) for (int k = 0; k < 4; ++k) P->kid[k].reset();
    for (QNode* a : refine) refine_node(a);
    st->coarsened = (int64_t)coarsen.size();
    st->refined = (int64_t)refine.size();
    relist();
    relocate_all();
    /* refine again while a leaf is over the upper bound */
    for (;;) {
      for (int sp = 0; sp < d.nspecies; ++sp) c[sp] = counts(sp);
      std::vector<QNode*> more;
      for (size_t l = 0; l < leaves.size(); ++l)
        if (nmax(c, l) > n_hi && leaves[l]->level < d.max_level) more.push_back(leaves[l]);
      if (more.empty()) break;
      for (QNode* a : more) refine_node(a);
      st->refined += (int64_t)more.size();
      relist();
      relocate_all();
    }
    st->balance_refined = balance();
    relist();
    relocate_all();
    int rc = split(n_lo, st);
    if (rc != OR_OK) return rc;
    merge(n_hi, st);
    st->nleaves = (int64_t)leaves.size();
    deposit();
    return OR_OK;
  }

  int split(int n_lo, or_adapt_stats* st) {
    for (;;) {
      std::vector<std::vector<int64_t>> c(d.nspecies);
      for (int sp = 0; sp < d.nspecies; ++sp) c[sp] = counts(sp);
      struct Par { uint32_t id; int sp; size_t idx; };
      std::vector<Par> par;
      for (int sp = 0; sp < d.nspecies; ++sp)
        for (size_t i = 0; i < p[sp].size(); ++i) {
          const Particle<T>& q = p[sp][i];
          int64_t n = c[sp][q.cell];
          if (n > 0 && n < n_lo && q.w % 4u == 0 && q.w >= 4u) par.push_back(Par{q.id, sp, i});
        }
      if (par.empty()) return OR_OK;
      std::sort(par.begin(), par.end(), [](const Par& a, const Par& b) { return a.id < b.id; });
      if ((uint64_t)next_id + 3ull * par.size() > 0xFFFFFFFFull) return OR_E_CAPACITY;
      std::vector<Particle<T>> add[2];
      for (size_t r = 0; r < par.size(); ++r) {
        Particle<T>& q = p[par[r].sp][par[r].idx];
        q.w /= 4u;
        for (uint32_t k = 0; k < 3; ++k) {
          Particle<T> cpy = q;
          cpy.id = next_id + 3u * (uint32_t)r + k;
          add[par[r].sp].push_back(cpy);
        }
      }
      next_id += 3u * (uint32_t)par.size();
      for (int sp = 0; sp < d.nspecies; ++sp) p[sp].insert(p[sp].end(), add[sp].begin(), add[sp].end());
      st->split_parents += (int64_t)par.size();
    }
  }

  void merge(int n_hi, or_adapt_stats* st) {
    for (int sp = 0; sp < d.nspecies; ++sp) {
      for (;;) {
        std::vector<int64_t> c = counts(sp);
        std::vector<std::vector<size_t>> grp(leaves.size());
        bool any = false;
        for (size_t i = 0; i < p[sp].size(); ++i) {
          int64_t l = p[sp][i].cell;
          if (c[l] > n_hi) { grp[l].push_back(i); any = true; }
        }
        if (!any) break;
        bool merged_any = false;
        for (size_t l = 0; l < leaves.size(); ++l) {
          std::vector<size_t>& g = grp[l];
          if (g.empty()) continue;
          std::vector<Particle<T>>& P = p[sp];
          auto oct = [](const Particle<T>& q) {
            return (q.v[0] < (T)0 ? 1 : 0) | (q.v[1] < (T)0 ? 2 : 0) | (q.v[2] < (T)0 ? 4 : 0);
          };
          auto v2 = [](const Particle<T>& q) { return (q.v[0] * q.v[0] + q.v[1] * q.v[1]) + q.v[2] * q.v[2]; };
          std::sort(g.begin(), g.end(), [&](size_t x, size_t y) {
            int ox = oct(P[x]), oy = oct(P[y]);
            if (ox != oy) return ox < oy;
            T ex = v2(P[x]), ey = v2(P[y]);
            if (ex != ey) return ex < ey;
            return P[x].id < P[y].id;
          });
          const QNode* lf = leaves[l];
          T lo[2] = {(T)lf->x0(), (T)lf->y0()};
          T hi[2] = {(T)lf->x1(), (T)lf->y1()};
          for (size_t k = 0; k + 1 < g.size(); k += 2) {
            Particle<T>& A = P[g[k]];
            Particle<T>& B = P[g[k + 1]];
            uint64_t ws = (uint64_t)A.w + (uint64_t)B.w;
            if (ws > 0xFFFFFFFFull) continue;
            double wa = (double)A.w, wb = (double)B.w, wt = (double)ws;
            double e_before = wa * ((double)v2(A)) + wb * ((double)v2(B));
            Particle<T>& keep = (A.id < B.id) ? A : B;
            Particle<T>& gone = (A.id < B.id) ? B : A;
            T ns[2], nv[3];
            for (int c2 = 0; c2 < 2; ++c2) {
              T x = (T)((wa * (double)A.s[c2] + wb * (double)B.s[c2]) / wt);
              if (x < lo[c2]) x = lo[c2];
              if (x >= hi[c2]) x = std::nextafter(hi[c2], (T)0);
              ns[c2] = x;
            }
            for (int c2 = 0; c2 < 3; ++c2) nv[c2] = (T)((wa * (double)A.v[c2] + wb * (double)B.v[c2]) / wt);
            keep.s[0] = ns[0]; keep.s[1] = ns[1];
            for (int c2 = 0; c2 < 3; ++c2) keep.v[c2] = nv[c2];
            keep.w = (uint32_t)ws;
            gone.alive = false;
            st->merge_energy_change += wt * (double)v2(keep) - e_before;
            st->merged_pairs++;
            merged_any = true;
          }
        }
        p[sp].erase(std::remove_if(p[sp].begin(), p[sp].end(), [](const Particle<T>& q) { return !q.alive; }),
                    p[sp].end());
        if (!merged_any) break;
      }
    }
  }

  int read(int species, double* s, double* v, uint32_t* w, uint32_t* id, uint32_t* cell) const {
    if (species < 0 || species >= d.nspecies) return OR_E_ARG;
    int dim = d.dim;
    for (size_t i = 0; i < p[species].size(); ++i) {
      const Particle<T>& q = p[species][i];
      for (int c = 0; c < dim; ++c) if (s) s[i * dim + c] = (double)q.s[c];
      for (int c = 0; c < 3; ++c) if (v) v[i * 3 + c] = (double)q.v[c];
      if (w) w[i] = q.w;
      if (id) id[i] = q.id;
      if (cell) {
        if (dim == 1) {
          T g = q.s[0] * (T)N;
          int64_t ic = (int64_t)std::floor(g);
          if (ic > N - 1) ic = N - 1;
          cell[i] = (uint32_t)ic;
        } else {
          cell[i] = (uint32_t)q.cell;
        }
      }
    }
    return OR_OK;
  }

  /* v^{-1/2} = v^0 - (q dt / 2m) E^0(x^0) */
  int leapfrog_start() {
    for (int sp = 0; sp < d.nspecies; ++sp) {
      const SpeciesK<T>& k = K[sp];
      for (Particle<T>& q : p[sp]) {
        if (d.dim == 1) {
          T E = gather1d(q.s[0]);
          q.v[0] = q.v[0] - k.hqm_dtT * E;
          q.b = d.field_scheme == OR_FIELD_DIPIC ? k.hqm_dtT * E : (T)0;   /* filtered acceleration a(x_0) */
        } else if (d.dim == 3) {
          T E[3];
          gather3d(q, E);
          for (int a = 0; a < 3; ++a) q.v[a] = q.v[a] - k.hqm_dtT * E[a];
        } else {
          T E[2];
          gather2d(q, E);
          q.v[0] = q.v[0] - k.hqm_dtT * E[0];
          q.v[1] = q.v[1] - k.hqm_dtT * E[1];
        }
      }
    }
    return OR_OK;
  }
};

template <class F> auto dispatch(void* h, F f) -> decltype(f(*(Sim<double>*)nullptr)) {
  SimBase* b = (SimBase*)h;
  if (b->d.precision == 32) return f(*(Sim<float>*)b);
  return f(*(Sim<double>*)b);
}

}  // namespace

extern "C" {

void or_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) { philox10<uint32_t>(ctr, key, out); }
void or_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) { philox10<uint64_t>(ctr, key, out); }

void* or_create(const or_desc* d) {
  if (!d || d->dim < 1 || d->dim > 3 || (d->precision != 32 && d->precision != 64) ||
      d->nspecies < 1 || d->nspecies > 2 || !(d->length > 0) || !(d->dt > 0) ||
      (d->field_scheme != OR_FIELD_CIC_EM && d->field_scheme != OR_FIELD_CIC_EC &&
       d->field_scheme != OR_FIELD_CIC_AMR && d->field_scheme != OR_FIELD_DIPIC) ||
      (d->dim >= 2 && d->field_scheme == OR_FIELD_CIC_EC) ||    /* energy-conserving: uniform 1D mesh */
      (d->dim == 1 && d->field_scheme == OR_FIELD_CIC_AMR) ||   /* cloud on the tree: 2D */
      (d->dim != 1 && d->field_scheme == OR_FIELD_DIPIC))       /* direct implicit: 1D */
    return nullptr;
  SimBase* b;
  bool ok;
  if (d->precision == 32) {
    Sim<float>* s = new Sim<float>();
    s->d = *d; ok = s->build(); b = s;
  } else {
    Sim<double>* s = new Sim<double>();
    s->d = *d; ok = s->build(); b = s;
  }
  if (!ok) { delete b; return nullptr; }
  return b;
}

void or_destroy(void* h) { delete (SimBase*)h; }

int or_load(void* h, int species, int64_t n, const double* s, const double* v, const uint32_t* w,
            const uint32_t* id) {
  return dispatch(h, [&](auto& S) { return S.load(species, n, s, v, w, id); });
}

int64_t or_count(void* h, int species) {
  return dispatch(h, [&](auto& S) { return (int64_t)S.p[species].size(); });
}

uint32_t or_next_id(void* h) { return dispatch(h, [&](auto& S) { return S.next_id; }); }

int or_read(void* h, int species, double* s, double* v, uint32_t* w, uint32_t* id, uint32_t* cell) {
  return dispatch(h, [&](auto& S) { return S.read(species, s, v, w, id, cell); });
}

int64_t or_nleaves(void* h) {
  return dispatch(h, [&](auto& S) { return S.d.dim == 3 ? (int64_t)S.leaves3.size() : (int64_t)S.leaves.size(); });
}

int or_leaves(void* h, uint32_t* keys, uint8_t* levels) {
  return dispatch(h, [&](auto& S) {
    if (S.d.dim == 3) {   /* keys: Morton codes of the 10-bit corner coordinates */
      for (size_t l = 0; l < S.leaves3.size(); ++l) {
        const ONode* n = S.leaves3[l];
        const uint32_t sh = 10 - n->level;
        keys[l] = morton10(n->i[0] << sh, n->i[1] << sh, n->i[2] << sh);
        levels[l] = (uint8_t)n->level;
      }
      return OR_OK;
    }
    for (size_t l = 0; l < S.leaves.size(); ++l) {
      const QNode* n = S.leaves[l];
      uint32_t sh = 16 - n->level;
      keys[l] = morton16(n->ix << sh, n->iy << sh);
      levels[l] = (uint8_t)n->level;
    }
    return OR_OK;
  });
}

int64_t or_nq(void* h) { return dispatch(h, [&](auto& S) { return S.nq(); }); }

int or_deposit(void* h, uint64_t* q_out) {
  return dispatch(h, [&](auto& S) {
    S.deposit();
    int64_t n = S.nq();
    if (q_out)
      for (int sp = 0; sp < 2; ++sp)
        for (int64_t i = 0; i < n; ++i) q_out[sp * n + i] = S.Q[sp][i];
    return OR_OK;
  });
}

int or_field_set(void* h, int kind, const double* data) {
  return dispatch(h, [&](auto& S) {
    using T = typename std::remove_reference<decltype(S.En)>::type::value_type;
    if (S.d.dim == 1) {
      const bool ec = S.d.field_scheme == OR_FIELD_CIC_EC;
      if (kind == OR_NODE_E_1D) {   /* node E: momentum-conserving coupling only */
        if (ec) return OR_E_ARG;
        for (int i = 0; i <= S.N; ++i) S.En[i] = (T)data[i];
        return OR_OK;
      }
      if (kind == OR_CELL_E_1D) {   /* cell E: energy-conserving coupling only */
        if (!ec) return OR_E_ARG;
        for (int i = 0; i < S.N; ++i) S.En[i] = (T)data[i];
        S.En[S.N] = (T)0;
        return OR_OK;
      }
      if (kind == OR_NODE_PHI_1D) {
        double inv2dx = 1.0 / (2.0 * (S.d.length / S.N));
        std::vector<double> e(S.N + 1);
        S.node_or_cell_e(data, inv2dx, e.data());
        for (int i = 0; i <= S.N; ++i) S.En[i] = (T)e[i];
        return OR_OK;
      }
      return OR_E_ARG;
    }
    if (S.d.dim == 3) {
      const size_t n3 = S.leaves3.size();
      if (kind == OR_CORNER_PHI_3D) {
        S.corner_field3(data);
        return OR_OK;
      }
      if (kind == OR_CORNER_E_3D) {
        for (size_t i = 0; i < n3 * 24; ++i) { S.cornerE3_64[i] = data[i]; S.cornerE3[i] = (T)data[i]; }
        return OR_OK;
      }
      return OR_E_ARG;
    }
    size_t nl = S.leaves.size();
    if (kind == OR_CORNER_PHI_2D) {
      std::vector<double> c(data, data + nl * 4);
      S.corner_field_from_corner_phi(c);
      return OR_OK;
    }
    if (kind == OR_CORNER_E_2D) {
      for (size_t i = 0; i < nl * 8; ++i) { S.cornerE64[i] = data[i]; S.cornerE[i] = (T)data[i]; }
      S.cell_e_from_corners();
      return OR_OK;
    }
    if (kind == OR_CELL_E_2D) {   /* the cloud-in-cell gather table, given directly */
      if (S.d.field_scheme != OR_FIELD_CIC_AMR) return OR_E_ARG;
      for (size_t i = 0; i < nl * 2; ++i) { S.cellE64[i] = data[i]; S.cellE[i] = (T)data[i]; }
      return OR_OK;
    }
    if (kind == OR_CELL_PHI_2D) {
      S.corner_field_from_cell_phi(data);
      return OR_OK;
    }
    return OR_E_ARG;
  });
}

int or_rho(void* h, double* rho_out) {
  return dispatch(h, [&](auto& S) {
    S.rho(rho_out);
    return OR_OK;
  });
}

int or_corner_phi(void* h, double* out) {
  return dispatch(h, [&](auto& S) {
    if (S.d.dim != 2) return (int)OR_E_ARG;
    for (size_t i = 0; i < S.cornerPhi.size(); ++i) out[i] = S.cornerPhi[i];
    return (int)OR_OK;
  });
}

int or_set_next_id(void* h, uint32_t next_id) {
  return dispatch(h, [&](auto& S) {
    for (int sp = 0; sp < S.d.nspecies; ++sp)
      for (const auto& q : S.p[sp])
        if (q.id >= next_id) return (int)OR_E_ARG;
    S.next_id = next_id;
    return (int)OR_OK;
  });
}

int or_field_table(void* h, double* out) {
  return dispatch(h, [&](auto& S) {
    if (S.d.dim == 1)
      for (int i = 0; i <= S.N; ++i) out[i] = (double)S.En[i];
    else if (S.d.dim == 3)
      for (size_t i = 0; i < S.cornerE3.size(); ++i) out[i] = (double)S.cornerE3[i];
    else if (S.d.field_scheme == OR_FIELD_CIC_AMR)
      for (size_t i = 0; i < S.cellE.size(); ++i) out[i] = (double)S.cellE[i];
    else
      for (size_t i = 0; i < S.cornerE.size(); ++i) out[i] = (double)S.cornerE[i];
    return OR_OK;
  });
}

int or_gather(void* h, int64_t n, const double* s, double* out) {
  return dispatch(h, [&](auto& S) {
    using T = typename std::remove_reference<decltype(S.En)>::type::value_type;
    for (int64_t i = 0; i < n; ++i) {
      if (S.d.dim == 1) {
        const T x = (T)s[i];
        if (!(x >= (T)0 && x < (T)1)) return (int)OR_E_ARG;
        out[i] = (double)S.gather1d(x);
      } else if (S.d.dim == 3) {
        Particle<T> q;
        for (int a = 0; a < 3; ++a) {
          q.s[a] = (T)s[3 * i + a];
          if (!(q.s[a] >= (T)0 && q.s[a] < (T)1)) return (int)OR_E_ARG;
        }
        q.cell = S.locate_cell(q.s);
        T E[3];
        S.gather3d(q, E);
        for (int a = 0; a < 3; ++a) out[3 * i + a] = (double)E[a];
      } else {
        Particle<T> q;
        q.s[0] = (T)s[2 * i];
        q.s[1] = (T)s[2 * i + 1];
        if (!(q.s[0] >= (T)0 && q.s[0] < (T)1 && q.s[1] >= (T)0 && q.s[1] < (T)1)) return (int)OR_E_ARG;
        q.cell = S.locate_cell(q.s);
        T E[2];
        S.gather2d(q, E);
        out[2 * i] = (double)E[0];
        out[2 * i + 1] = (double)E[1];
      }
    }
    return (int)OR_OK;
  });
}

int or_field_solve_1d(void* h, double phi_left, double* phi_out, double* e_out) {
  return dispatch(h, [&](auto& S) {
    if (S.d.dim != 1) return (int)OR_E_ARG;
    S.solve1d(phi_left, phi_out, e_out);
    return (int)OR_OK;
  });
}

int or_dipic_field(void* h, double phi_left, double* phi_out, double* chi_out) {
  return dispatch(h, [&](auto& S) {
    if (S.d.dim != 1 || S.d.field_scheme != OR_FIELD_DIPIC) return (int)OR_E_ARG;
    S.deposit();
    S.solve1d_implicit(phi_left, phi_out, chi_out);
    return (int)OR_OK;
  });
}

int or_field_solve_2d(void* h, const double* phi_init, double rtol, int maxit, double* phi_out, int* iters,
                      double* relres) {
  return dispatch(h, [&](auto& S) {
    if (S.d.dim != 2) return (int)OR_E_ARG;
    return S.cg2d(phi_init, rtol, maxit, phi_out, iters, relres);
  });
}

int64_t or_assemble_2d(void* h, int32_t* rows, int32_t* cols, double* vals, double* rhs) {
  return dispatch(h, [&](auto& S) {
    if (S.d.dim != 2) return (int64_t)-1;
    std::vector<typename std::remove_reference<decltype(S)>::type::Row> R;
    S.assemble(R);
    int64_t k = 0;
    for (size_t i = 0; i < R.size(); ++i) {
      if (rows) { rows[k] = (int32_t)i; cols[k] = (int32_t)i; vals[k] = R[i].diag; }
      ++k;
      for (auto& e : R[i].off) {
        if (rows) { rows[k] = (int32_t)i; cols[k] = (int32_t)e.first; vals[k] = -e.second; }
        ++k;
      }
      if (rhs) rhs[i] = S.rhs_cell(i) + R[i].bnd;
    }
    return k;
  });
}

int or_leapfrog_start(void* h) {
  return dispatch(h, [&](auto& S) { return S.leapfrog_start(); });
}

int or_step(void* h, int64_t step0, int nsteps, const double* v_next, int solve_1d, or_stats* st) {
  std::memset(st, 0, sizeof(*st));
  return dispatch(h, [&](auto& S) {
    if (S.d.field_scheme == OR_FIELD_DIPIC && !solve_1d) return (int)OR_E_ARG;   /* the field is part of the step */
    for (int k = 0; k < nsteps; ++k) {
      if (S.d.field_scheme == OR_FIELD_DIPIC) {
        int rc = S.step_dipic((uint32_t)(step0 + k), v_next[k], st);
        if (rc != OR_OK) return rc;
        continue;
      }
      int rc = S.step((uint32_t)(step0 + k), st);
      if (rc != OR_OK) return rc;
      if (solve_1d && S.d.dim == 1) S.solve1d(v_next[k], nullptr, nullptr);
    }
    return (int)OR_OK;
  });
}

int or_adapt(void* h, int n_lo, int n_hi, or_adapt_stats* st) {
  return dispatch(h, [&](auto& S) {
    if (S.d.dim != 2) return (int)OR_E_ARG;
    return S.adapt(n_lo, n_hi, st);
  });
}

int or_locate(void* h, int64_t n, const double* s, uint32_t* leaf) {
  return dispatch(h, [&](auto& S) {
    if (S.d.dim == 3) {
      for (int64_t i = 0; i < n; ++i) leaf[i] = (uint32_t)locate3(S.root3.get(), &s[3 * i])->leaf_index;
      return (int)OR_OK;
    }
    if (S.d.dim != 2) return (int)OR_E_ARG;
    for (int64_t i = 0; i < n; ++i) leaf[i] = (uint32_t)locate_node(S.root.get(), s[2 * i], s[2 * i + 1])->leaf_index;
    return (int)OR_OK;
  });
}

void or_derived(void* h, int species, double* out) {
  dispatch(h, [&](auto& S) {
    auto& k = S.K[species];
    double v[] = {(double)k.qm_dtT, (double)k.dt_LT, (double)k.Tcand, (double)k.a_elT, (double)k.a_izT,
                  (double)k.v_iz2T, (double)k.mu2T, (double)k.vmax2T, (double)k.v_thgT, (double)k.a_cxT,
                  (double)k.gmaxT, (double)k.hqm_dtT};
    for (int i = 0; i < 12; ++i) out[i] = v[i];
    return 0;
  });
}

}  // extern "C"
