// Field kernels (FP64): the Poisson solves of the ES-PIC step and the tables
// the particle gather reads (arXiv:1604.07713, Sec. 3: potential at cell
// centres, E at cell nodes/corners, bilinear gather).
//
//  1D: one workgroup per instance: the exact solution of the node system
//      through the closed-form inverse of tridiag(-1,2,-1), with 128-bit
//      integer prefix sums of the charge sums (no sequential sweep); node E
//      by centred differences inside, second-order one-sided at the walls.
//  2D: cell-centred finite volumes on the leaves with two-point fluxes,
//      solved by Jacobi-preconditioned CG; node potentials are the mean of
//      the cell potentials of the leaves having the node as a corner
//      (Dirichlet wall value on the walls), and nodal E the mean of those
//      leaves' corner gradients.
#include "device_util.hpp"
#include "pic_internal.hpp"

namespace pic {

// ---------------------------------------------------------------------------
// 1D
// ---------------------------------------------------------------------------
// The exact solution of the 1D node system 2 phi_i - phi_{i-1} - phi_{i+1} =
// c_i (i = 1..N-1, phi_0 = V, phi_N = 0, c_i = sum_s kappa_s Q_s,i) through
// the inverse of tridiag(-1, 2, -1), (A^-1)_ij = min(i,j) (N - max(i,j)) / N:
//   phi_i = V (N - i) / N + sum_s (kappa_s / N) D_s,i,
//   D_s,i = (N - i) sum_{j<=i} j Q_s,j + i sum_{j>i} (N - j) Q_s,j.
// D is an exact integer (the Q are integer charge sums): each thread sums its
// run of nodes in 128-bit integers, a workgroup scan gives every node its
// prefix sums, and D is rounded to double once.  The result does not depend
// on how the nodes are split between threads, so it is the same for every
// launch shape, and it is the exact solution rounded (a few ulps of its
// terms) instead of a sequential sweep's rounding.
typedef unsigned __int128 u128;

__device__ __forceinline__ u128 shfl_up_u128(u128 v, unsigned off) {
  const unsigned long long lo = (unsigned long long)v, hi = (unsigned long long)(v >> 64);
  const unsigned long long l2 = __shfl_up(lo, off), h2 = __shfl_up(hi, off);
  return ((u128)h2 << 64) | (u128)l2;
}

constexpr int kField1dThreads = 1024;

template <class T>
__global__ __launch_bounds__(kField1dThreads) void k_field1d(const InstDev<T>* __restrict__ insts, int mode,
                                                             const double* __restrict__ phi_left) {
  extern __shared__ double ph[];   // [N + 1] node potentials
  __shared__ u128 wtot[kField1dThreads / 64][4];
  const InstDev<T>& I = insts[blockIdx.x];
  // after a step that was not run for want of room, neither solve nor commit
  // (the table keeps the field of the last committed step)
  if (mode == 1 && (I.ctr->flags & kFlagNeedRoom)) return;
  const int N = I.N;
  const uint32_t step = I.ctr->step;
  const uint32_t par = mode == 1 ? (step & 1u) : ((step + 1u) & 1u);
  const unsigned long long* Q = I.Q + (size_t)par * 2u * I.nq;
  double left;
  if (mode == 1) {
    const uint32_t k = step + 1u - I.ctr->vstep0;
    left = (I.v_table && k < I.v_len) ? I.v_table[k] : 0.0;
  } else {
    left = phi_left ? phi_left[blockIdx.x] : 0.0;
  }
  // interior nodes [j0, j1) of this thread
  const int per = (N - 1 + (int)blockDim.x - 1) / (int)blockDim.x;
  const int j0 = 1 + (int)threadIdx.x * per;
  const int j1 = j0 + per < N ? j0 + per : N;
  const int ns = I.nspecies;
  // q[0..1]: sum j Q_s,j and sum (N - j) Q_s,j of species 0; q[2..3] of species 1
  // (species loops unrolled with constant indices: the arrays stay in registers)
  u128 q[4] = {0, 0, 0, 0};
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
    if (sp >= ns) break;
    for (int j = j0; j < j1; ++j) {
      const u128 v = (u128)Q[(size_t)sp * I.nq + j];
      q[2 * sp] += (u128)(unsigned)j * v;
      q[2 * sp + 1] += (u128)(unsigned)(N - j) * v;
    }
  }
  // workgroup exclusive scan of the four sums (inclusive within the wave by
  // shuffles, then the totals of the lower waves)
  const int lane = lane_id(), wv = threadIdx.x / 64, nw = blockDim.x / 64;
  u128 inc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    inc[k] = q[k];
#pragma unroll
    for (unsigned off = 1; off < 64; off <<= 1) {
      const u128 o = shfl_up_u128(inc[k], off);
      if (lane >= (int)off) inc[k] += o;
    }
  }
  if (lane == 63)
#pragma unroll
    for (int k = 0; k < 4; ++k) wtot[wv][k] = inc[k];
  __syncthreads();
  u128 base[4] = {0, 0, 0, 0}, total[4] = {0, 0, 0, 0};
  for (int w = 0; w < nw; ++w) {
    const bool lower = w < wv;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const u128 t = wtot[w][k];
      base[k] += lower ? t : (u128)0;
      total[k] += t;
    }
  }
  // the thread's nodes: prefix sums through node j, then D and phi
  u128 P[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) P[k] = base[k] + inc[k] - q[k];
  const double dN = (double)N;
  for (int j = j0; j < j1; ++j) {
    double v = (left * (double)(N - j)) / dN;
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      if (sp >= ns) break;
      const u128 qq = (u128)Q[(size_t)sp * I.nq + j];
      P[2 * sp] += (u128)(unsigned)j * qq;
      P[2 * sp + 1] += (u128)(unsigned)(N - j) * qq;
      const u128 D = (u128)(unsigned)(N - j) * P[2 * sp] + (u128)(unsigned)j * (total[2 * sp + 1] - P[2 * sp + 1]);
      v = v + ((double)D * I.kappa[sp]) / dN;
    }
    ph[j] = v;
  }
  if (threadIdx.x == 0) {
    ph[0] = left;
    ph[N] = 0.0;
  }
  __syncthreads();
  T* E = const_cast<T*>(I.E);
  const double h2 = I.inv2dx;
  for (int i = threadIdx.x; i <= N; i += blockDim.x) {
    double e;
    if (I.cell_e) e = i < N ? (ph[i] - ph[i + 1]) * (2.0 * h2) : 0.0;   // cell E (energy-conserving)
    else if (i == 0) e = ((3.0 * ph[0] - 4.0 * ph[1]) + ph[2]) * h2;
    else if (i == N) e = ((-3.0 * ph[N] + 4.0 * ph[N - 1]) - ph[N - 2]) * h2;
    else e = (ph[i - 1] - ph[i + 1]) * h2;
    E[i] = (T)e;
    if (I.e64) I.e64[i] = e;
    if (I.phi64) I.phi64[i] = ph[i];
  }
  if (mode == 1 && threadIdx.x == 0) {
    // commit the step: births join the counts, the step index advances
    Counters* c = I.ctr;
    const uint32_t nb = c->nbirths;
    if (nb && !(c->flags & (kFlagBirthOverflow | kFlagIdOverflow))) {
      c->count[0] += nb;
      c->count[1] += nb;
      c->next_id += 2u * nb;
      c->stats[kStBirths] += nb;
    }
    c->nbirths = 0u;
    c->step = step + 1u;
  }
}

template <class T>
hipError_t launch_field1d(const InstDev<T>* insts, int ninst, int max_n, int mode, const double* phi_left,
                          hipStream_t s) {
  const size_t lds = (size_t)(max_n + 1) * sizeof(double);
  hipLaunchKernelGGL(k_field1d<T>, dim3(ninst), dim3(kField1dThreads), lds, s, insts, mode, phi_left);
  return hipGetLastError();
}

// Direct implicit field (Sec. 3, D1 scheme): one workgroup.  The charge of
// the predicted positions (Qp) gives the susceptibility at the nodes, chi_i
// = sum_s chi_s Qp_s,i (a wall node's charge fills half a cell: twice
// that), and the right-hand side c_i = sum_s kappa_s Qp_s,i; the node system
//   -f_i-1 phi_i-1 + (f_i-1 + f_i) phi_i - f_i phi_i+1 = c_i  (i = 1..N-1),
//   f_i = 1 + (chi_i + chi_i+1)/2,  phi_0 = V (the next drive value), phi_N = 0,
// is solved by forward elimination and back substitution.  The recurrences
// are sequential (one lane, FP64 divisions); the workgroup forms the face
// coefficients and right-hand sides of a chunk of nodes straight from Qp
// into LDS ahead of the lane's sweep, which also stores c', d' to the
// scratch dws [3][N+1] (read back only by meshes beyond one chunk).  With
// N <= kDipicChunk phi stays in LDS, else it goes to dws too.  Node E as in the explicit solve; Qp is cleared for the next
// step.
constexpr int kDipicThreads = 1024;
constexpr int kDipicChunk = 1920;

template <class T>
__device__ __forceinline__ double dipic_chi(const InstDev<T>& I, const unsigned long long* Qp, int i) {
  double c = 0.0;
  for (int sp = 0; sp < I.nspecies; ++sp) c = c + I.chi[sp] * (double)(long long)Qp[(size_t)sp * I.nq + i];
  return (i == 0 || i == I.N) ? 2.0 * c : c;   // a wall node's charge fills half a cell
}
template <class T>
__device__ __forceinline__ double dipic_face(const InstDev<T>& I, const unsigned long long* Qp, int i) {
  return 1.0 + (dipic_chi<T>(I, Qp, i) + dipic_chi<T>(I, Qp, i + 1)) * 0.5;   // face i + 1/2
}

template <class T>
__global__ __launch_bounds__(kDipicThreads) void k_dipic_field(InstDev<T> I) {
  __shared__ double sf[kDipicChunk + 1], sr[kDipicChunk], scp[kDipicChunk], sdp[kDipicChunk];
  if (I.ctr->flags & kFlagNeedRoom) return;   // the predictor did not run this step
  const int N = I.N;
  const uint32_t nq = I.nq;
  const int tid = threadIdx.x, nt = blockDim.x;
  const uint32_t kk = I.ctr->step + 1u - I.ctr->vstep0;
  const double left = (I.v_table && kk < I.v_len) ? I.v_table[kk] : 0.0;
  const bool single = N <= kDipicChunk;
  double* cp = I.dws;
  double* dp = I.dws + nq;
  double* ph = single ? sf : I.dws + 2u * nq;   // sf is free once the sweep is done
  unsigned long long* Qp = I.Qp;
  // forward elimination over chunks of nodes [c0, c0 + n); lane 0 carries
  // c', d' of the previous node
  double cprev = 0.0, dprev = 0.0;
  for (int c0 = 1; c0 < N; c0 += kDipicChunk) {
    const int n = N - c0 < kDipicChunk ? N - c0 : kDipicChunk;
    for (int t = tid; t <= n; t += nt) sf[t] = dipic_face<T>(I, Qp, c0 - 1 + t);
    for (int t = tid; t < n; t += nt) {
      const int i = c0 + t;
      double r = 0.0;
      for (int sp = 0; sp < I.nspecies; ++sp) r = r + (double)(long long)Qp[(size_t)sp * nq + i] * I.kappa[sp];
      if (i == 1) r = r + dipic_face<T>(I, Qp, 0) * left;
      sr[t] = r;
    }
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      if (c0 == 1) {   // node 1 starts the elimination
        const double bb = sf[0] + sf[1], c = -sf[1];
        cprev = c / bb;
        dprev = sr[0] / bb;
        scp[0] = cprev;
        sdp[0] = dprev;
        cp[1] = cprev;
        dp[1] = dprev;
        t = 1;
      }
      // branch-free body: the LDS operands of later nodes load ahead, the
      // two divisions of a node are independent
#pragma unroll 4
      for (; t < n; ++t) {
        const double a = -sf[t], bb = sf[t] + sf[t + 1], c = -sf[t + 1], r = sr[t];
        const double m = bb - a * cprev;
        const double cpi = c / m;
        const double dpi = (r - a * dprev) / m;
        scp[t] = cpi;
        sdp[t] = dpi;
        cp[c0 + t] = cpi;
        dp[c0 + t] = dpi;
        cprev = cpi;
        dprev = dpi;
      }
    }
    __syncthreads();
  }
  // the charge of the predicted positions is consumed
  for (uint32_t j = tid; j < (uint32_t)I.nspecies * nq; j += nt) Qp[j] = 0ull;
  // back substitution over the same chunks from the top; the last chunk's
  // c', d' are still in LDS
  const int last = 1 + ((N - 2) / kDipicChunk) * kDipicChunk;
  double next = 0.0;
  for (int c0 = last; c0 >= 1; c0 -= kDipicChunk) {
    const int n = N - c0 < kDipicChunk ? N - c0 : kDipicChunk;
    if (c0 != last) {
      for (int t = tid; t < n; t += nt) {
        scp[t] = cp[c0 + t];
        sdp[t] = dp[c0 + t];
      }
    }
    __syncthreads();
    if (tid == 0) {
      int t = n - 1;
      if (c0 == last) {   // node N - 1
        next = sdp[t];
        ph[c0 + t] = next;
        --t;
      }
#pragma unroll 4
      for (; t >= 0; --t) {
        next = sdp[t] - scp[t] * next;
        ph[c0 + t] = next;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    ph[0] = left;
    ph[N] = 0.0;
  }
  __syncthreads();
  T* E = const_cast<T*>(I.E);
  const double h2 = I.inv2dx;
  for (int i = tid; i <= N; i += nt) {
    double e;
    if (i == 0) e = ((3.0 * ph[0] - 4.0 * ph[1]) + ph[2]) * h2;
    else if (i == N) e = ((-3.0 * ph[N] + 4.0 * ph[N - 1]) - ph[N - 2]) * h2;
    else e = (ph[i - 1] - ph[i + 1]) * h2;
    E[i] = (T)e;
    if (I.e64) I.e64[i] = e;
    if (I.phi64) I.phi64[i] = ph[i];
  }
}

template <class T>
hipError_t launch_dipic_field(const InstDev<T>& I, hipStream_t s) {
  hipLaunchKernelGGL(k_dipic_field<T>, dim3(1), dim3(kDipicThreads), 0, s, I);
  return hipGetLastError();
}

// Charge density of an integer deposit (Sec. 3: charge at the nodes of the
// uniform mesh or the centres of the leaves; Sec. 3.1: no per-level volume
// weighting): the sums scaled to coulombs (w_units = 2^16 carries w0 real
// particles, 1D shares carry F more bits), over dx (1D, per unit area) or
// over h^2 depth_z (2D), species added in order.
__global__ void k_rho(const unsigned long long* Q, uint32_t nq, int nspecies, double qw0_0, double qw0_1, int shift,
                      double dx, const uint8_t* lv, double length, double depth_z, int cube, double* rho) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  double r = 0.0;
  for (int sp = 0; sp < nspecies; ++sp) {
    const double units = (double)(long long)Q[(size_t)sp * nq + i];
    const double qw0 = sp == 0 ? qw0_0 : qw0_1;
    if (!lv) {
      r = r + ((units * ldexp(1.0, -shift)) * qw0) / dx;
    } else {
      const double h = length * ldexp(1.0, -(int)lv[i]);
      r = r + ((units * ldexp(1.0, -shift)) * qw0) / ((h * h) * (cube ? h : depth_z));
    }
  }
  rho[i] = r;
}

hipError_t launch_rho(const unsigned long long* Q, uint32_t nq, int nspecies, double qw0_0, double qw0_1, int shift,
                      double dx, const uint8_t* lv, double length, double depth_z, int cube, double* rho,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_rho, dim3(ceil_div(nq, kBlock)), dim3(kBlock), 0, s, Q, nq, nspecies, qw0_0, qw0_1, shift, dx,
                     lv, length, depth_z, cube, rho);
  return hipGetLastError();
}

// node E (or node potential -> E) given by the caller, rounded to T; with
// the energy-conserving coupling the table holds cell E (N values, then 0)
template <class T>
__global__ void k_node_e_1d(T* E, double* e64, const double* data, int is_phi, int N, double inv2dx, int cell_e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > N) return;
  double e;
  if (!is_phi) {
    e = data[i];
  } else if (cell_e) {
    e = i < N ? (data[i] - data[i + 1]) * (2.0 * inv2dx) : 0.0;
  } else if (i == 0) {
    e = ((3.0 * data[0] - 4.0 * data[1]) + data[2]) * inv2dx;
  } else if (i == N) {
    e = ((-3.0 * data[N] + 4.0 * data[N - 1]) - data[N - 2]) * inv2dx;
  } else {
    e = (data[i - 1] - data[i + 1]) * inv2dx;
  }
  E[i] = (T)e;
  if (e64) e64[i] = e;
}

template <class T>
hipError_t launch_node_e_1d(const InstDev<T>& I, const double* data, int is_phi, hipStream_t s) {
  hipLaunchKernelGGL(k_node_e_1d<T>, dim3(ceil_div(I.N + 1, kBlock)), dim3(kBlock), 0, s, const_cast<T*>(I.E),
                     I.e64, data, is_phi, I.N, I.inv2dx, I.cell_e);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 2D: nodes, corner gradients, nodal E
// ---------------------------------------------------------------------------
struct LeafBox {
  uint32_t x0, y0, size;
};
__device__ __forceinline__ LeafBox leaf_box(const Mesh2D& m, uint32_t l) {
  const uint32_t xy = m.xy[l];
  return LeafBox{xy >> 16, xy & 0xFFFFu, 1u << (16 - m.lv[l])};
}

// Leaves having node (X, Y) as a corner, in quadrant order SW, SE, NW, NE;
// returns their count and, per entry, the leaf and the corner index of the
// node in that leaf (0 = low-low, 1 = high x, 2 = high y, 3 = high-high).
__device__ __forceinline__ int node_leaves(const Mesh2D& m, uint32_t X, uint32_t Y, uint32_t* leaf, int* corner) {
  int k = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int qx = q & 1, qy = q >> 1;        // 0: the quadrant below/left of the node
    if ((qx == 0 && X == 0u) || (qx == 1 && X >= 65536u)) continue;
    if ((qy == 0 && Y == 0u) || (qy == 1 && Y >= 65536u)) continue;
    const uint32_t px = qx ? X : X - 1u, py = qy ? Y : Y - 1u;
    const uint32_t l = locate_leaf(m.key, m.lv, m.lut, m.lut_level, px, py);
    const LeafBox b = leaf_box(m, l);
    if ((X & (b.size - 1u)) != 0u || (Y & (b.size - 1u)) != 0u) continue;   // node on an edge, not a corner
    leaf[k] = l;
    corner[k] = (qx ? 0 : 1) + (qy ? 0 : 2);
    ++k;
  }
  return k;
}

__device__ __forceinline__ bool dirichlet_node(const Mesh2D& m, uint32_t X, uint32_t Y, double& v) {
  if (X == 0u && m.field_bc[0] == PIC_WALL_DIRICHLET) { v = m.wall_phi[0]; return true; }
  if (X == 65536u && m.field_bc[1] == PIC_WALL_DIRICHLET) { v = m.wall_phi[1]; return true; }
  if (Y == 0u && m.field_bc[2] == PIC_WALL_DIRICHLET) { v = m.wall_phi[2]; return true; }
  if (Y == 65536u && m.field_bc[3] == PIC_WALL_DIRICHLET) { v = m.wall_phi[3]; return true; }
  return false;
}

__global__ void k_cell_to_corner_phi(Mesh2D m, const double* __restrict__ cell_phi, double* __restrict__ corner_phi) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4u * m.nleaves) return;
  const uint32_t l = t >> 2;
  const int c = (int)(t & 3u);
  const LeafBox b = leaf_box(m, l);
  const uint32_t X = b.x0 + ((c & 1) ? b.size : 0u), Y = b.y0 + ((c >> 1) ? b.size : 0u);
  double v;
  if (!dirichlet_node(m, X, Y, v)) {
    uint32_t lf[4];
    int cr[4];
    const int k = node_leaves(m, X, Y, lf, cr);
    double s = 0.0;
    for (int j = 0; j < k; ++j) s = s + cell_phi[lf[j]];
    v = s / (double)k;
  }
  corner_phi[t] = v;
}

hipError_t launch_cell_to_corner_phi(const Mesh2D& m, const double* cell_phi, double* corner_phi, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_to_corner_phi, dim3(ceil_div(4u * m.nleaves, kBlock)), dim3(kBlock), 0, s, m, cell_phi,
                     corner_phi);
  return hipGetLastError();
}

__global__ void k_corner_grad(Mesh2D m, const double* __restrict__ cphi, double* __restrict__ grad) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= m.nleaves) return;
  const double h = ldexp(m.length, -(int)m.lv[l]);
  const double* f = cphi + (size_t)l * 4u;
  double* g = grad + (size_t)l * 8u;
  for (int c = 0; c < 4; ++c) {
    const int a = c & 1, bb = c >> 1;
    g[c * 2 + 0] = (f[0 + 2 * bb] - f[1 + 2 * bb]) / h;
    g[c * 2 + 1] = (f[a + 0] - f[a + 2]) / h;
  }
}

template <class T>
__global__ void k_nodal_e(Mesh2D m, const double* __restrict__ grad, double* __restrict__ ce64, T* __restrict__ ce) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4u * m.nleaves) return;
  const uint32_t l = t >> 2;
  const int c = (int)(t & 3u);
  const LeafBox b = leaf_box(m, l);
  const uint32_t X = b.x0 + ((c & 1) ? b.size : 0u), Y = b.y0 + ((c >> 1) ? b.size : 0u);
  uint32_t lf[4];
  int cr[4];
  const int k = node_leaves(m, X, Y, lf, cr);
  double sx = 0.0, sy = 0.0;
  for (int j = 0; j < k; ++j) {
    sx = sx + grad[(size_t)lf[j] * 8u + cr[j] * 2 + 0];
    sy = sy + grad[(size_t)lf[j] * 8u + cr[j] * 2 + 1];
  }
  const double ex = sx / (double)k, ey = sy / (double)k;
  ce64[(size_t)t * 2u + 0] = ex;
  ce64[(size_t)t * 2u + 1] = ey;
  ce[(size_t)t * 2u + 0] = (T)ex;
  ce[(size_t)t * 2u + 1] = (T)ey;
}

template <class T>
hipError_t launch_corner_field(const Mesh2D& m, const double* corner_phi, double* grad, double* corner_e64, T* corner_e,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_corner_grad, dim3(ceil_div(m.nleaves, kBlock)), dim3(kBlock), 0, s, m, corner_phi, grad);
  hipLaunchKernelGGL(k_nodal_e<T>, dim3(ceil_div(4u * m.nleaves, kBlock)), dim3(kBlock), 0, s, m, grad, corner_e64,
                     corner_e);
  return hipGetLastError();
}

// ---- octree (3D): nodal E from potentials at each leaf's corners ----
// Corner c = a + 2b + 4e along x, y, z.  Each leaf's E = -grad of its
// trilinear potential at each corner; a node's E is the mean over the
// leaves having it as a corner, taken in octant order (below the node in x
// first, then y, then z), each octant's leaf found at the finest cell
// beside the node (Sec. 3: nodal E).  m.xy holds the packed 10-bit corner
// coordinates.
__global__ void k_corner_grad3(Mesh2D m, const double* __restrict__ cphi, double* __restrict__ grad) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= m.nleaves) return;
  const double h = ldexp(m.length, -(int)m.lv[l]);
  const double* f = cphi + (size_t)l * 8u;
  double* g = grad + (size_t)l * 24u;
  for (int c = 0; c < 8; ++c) {
    const int a = c & 1, b = (c >> 1) & 1, e = c >> 2;
    g[c * 3 + 0] = (f[0 + 2 * b + 4 * e] - f[1 + 2 * b + 4 * e]) / h;
    g[c * 3 + 1] = (f[a + 0 + 4 * e] - f[a + 2 + 4 * e]) / h;
    g[c * 3 + 2] = (f[a + 2 * b + 0] - f[a + 2 * b + 4]) / h;
  }
}

template <class T>
__global__ void k_nodal_e3(Mesh2D m, const double* __restrict__ grad, double* __restrict__ ce64,
                           T* __restrict__ ce) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 8u * m.nleaves) return;
  const uint32_t l = t >> 3;
  const int c = (int)(t & 7u);
  const uint32_t p = m.xy[l];
  const uint32_t size = 1u << (10 - (int)m.lv[l]);
  uint32_t X[3];
  for (int a = 0; a < 3; ++a) X[a] = ((p >> (10 * a)) & 0x3FFu) + (((c >> a) & 1) ? size : 0u);
  double sum[3] = {0.0, 0.0, 0.0};
  int k = 0;
  for (int q = 0; q < 8; ++q) {
    bool inside = true;
    uint32_t P[3];
    for (int a = 0; a < 3; ++a) {
      const int up = (q >> a) & 1;
      if ((up == 0 && X[a] == 0u) || (up == 1 && X[a] >= 1024u)) inside = false;
      P[a] = up ? X[a] : X[a] - 1u;
    }
    if (!inside) continue;
    const uint32_t leaf = locate_leaf3(m.key, m.lv, m.lut, m.lut_level, P[0], P[1], P[2]);
    const uint32_t ms = 1u << (10 - (int)m.lv[leaf]);
    if ((X[0] & (ms - 1u)) || (X[1] & (ms - 1u)) || (X[2] & (ms - 1u))) continue;   // not a corner of it
    int mc = 0;
    for (int a = 0; a < 3; ++a)
      if (!((q >> a) & 1)) mc |= 1 << a;   // the leaf lies below the node along a
    for (int a = 0; a < 3; ++a) sum[a] = sum[a] + grad[(size_t)leaf * 24u + mc * 3 + a];
    ++k;
  }
  for (int a = 0; a < 3; ++a) {
    const double e = sum[a] / (double)k;
    ce64[(size_t)t * 3u + a] = e;
    ce[(size_t)t * 3u + a] = (T)e;
  }
}

template <class T>
hipError_t launch_corner_field3(const Mesh2D& m, const double* corner_phi, double* grad, double* corner_e64,
                                T* corner_e, hipStream_t s) {
  hipLaunchKernelGGL(k_corner_grad3, dim3(ceil_div(m.nleaves, kBlock)), dim3(kBlock), 0, s, m, corner_phi, grad);
  hipLaunchKernelGGL(k_nodal_e3<T>, dim3(ceil_div(8u * m.nleaves, kBlock)), dim3(kBlock), 0, s, m, grad,
                     corner_e64, corner_e);
  return hipGetLastError();
}

template <class T>
__global__ void k_round(const double* src, T* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (T)src[i];
}
template <class T>
hipError_t launch_round_table(const double* src, T* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_round<T>, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, src, dst, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 2D finite-volume operator on the leaves
// ---------------------------------------------------------------------------
// Face coefficient min(h_a, h_b) / ((h_a + h_b) / 2) of a 2:1 tree: 1 between
// leaves of one level, the double nearest 2/3 between leaves one level apart
// (the quotient of exact binary fractions, whatever the levels).
constexpr double kFaceTwoThirds = 2.0 / 3.0;
__device__ __forceinline__ uint32_t face_code(double c, uint32_t* bad) {
  if (c == 1.0) return 1u;
  if (c == kFaceTwoThirds) return 2u;
  *bad = 1u;
  return 0u;
}
__device__ __forceinline__ double face_coef(uint32_t k) { return k == 1u ? 1.0 : (k == 2u ? kFaceTwoThirds : 0.0); }

__global__ void k_build_stencil(Mesh2D m, Stencil2D st) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= m.nleaves) return;
  const LeafBox b = leaf_box(m, l);
  const int la = m.lv[l];
  const double ha = ldexp(1.0, -la);
  uint32_t* nb = st.nbr + (size_t)l * 8u;
  uint32_t code = 0u;
  int k = 0;
  double diag = 0.0, bnd = 0.0;
  const uint32_t half = b.size >> 1;
  // sides: 0 west, 1 east, 2 south, 3 north
  for (int side = 0; side < 4; ++side) {
    bool wall;
    uint32_t p1x, p1y, p2x, p2y;
    switch (side) {
      case 0: wall = b.x0 == 0u; p1x = b.x0 - 1u; p1y = b.y0; p2x = p1x; p2y = b.y0 + half; break;
      case 1: wall = b.x0 + b.size >= 65536u; p1x = b.x0 + b.size; p1y = b.y0; p2x = p1x; p2y = b.y0 + half; break;
      case 2: wall = b.y0 == 0u; p1x = b.x0; p1y = b.y0 - 1u; p2x = b.x0 + half; p2y = p1y; break;
      default: wall = b.y0 + b.size >= 65536u; p1x = b.x0; p1y = b.y0 + b.size; p2x = b.x0 + half; p2y = p1y; break;
    }
    if (wall) {
      if (m.field_bc[side] == PIC_WALL_DIRICHLET) {
        diag = diag + 2.0;
        bnd = bnd + 2.0 * m.wall_phi[side];
      }
      continue;
    }
    const uint32_t n1 = locate_leaf(m.key, m.lv, m.lut, m.lut_level, p1x, p1y);
    const int l1 = m.lv[n1];
    const double h1 = ldexp(1.0, -l1);
    const double c1 = fmin(ha, h1) / ((ha + h1) / 2.0);
    nb[k] = n1;
    code |= face_code(c1, st.code + m.nleaves) << (2 * k);
    ++k;
    diag = diag + c1;
    if (l1 > la) {   // two finer neighbours share this side
      const uint32_t n2 = locate_leaf(m.key, m.lv, m.lut, m.lut_level, p2x, p2y);
      const double h2 = ldexp(1.0, -(int)m.lv[n2]);
      const double c2 = fmin(ha, h2) / ((ha + h2) / 2.0);
      nb[k] = n2;
      code |= face_code(c2, st.code + m.nleaves) << (2 * k);
      ++k;
      diag = diag + c2;
    }
  }
  for (; k < 8; ++k) nb[k] = l;
  st.code[l] = code;
  st.diag[l] = diag;
  st.bnd[l] = bnd;
}

hipError_t launch_build_stencil(const Mesh2D& m, const Stencil2D& st, hipStream_t s) {
  hipLaunchKernelGGL(k_build_stencil, dim3(ceil_div(m.nleaves, kBlock)), dim3(kBlock), 0, s, m, st);
  return hipGetLastError();
}

// CG with one global reduction per iteration (the Chronopoulos-Gear form of
// Jacobi-preconditioned CG: mathematically the same iterates as the textbook
// form).  With u = r / diag and w = A u, iteration k forms
//   s_k = w_k + beta_k s_{k-1},  p_k = u_k + beta_k p_{k-1},
//   x_{k+1} = x_k + alpha_k p_k,  r_{k+1} = r_k - alpha_k s_k,
//   w_{k+1} = A u_{k+1},
// and the three dot products r.u, w.u and r.r of the new vectors in one
// pass; beta_k = g_k / g_{k-1} and alpha_k = g_k / (d_k - beta_k g_k /
// alpha_{k-1}) with g = r.u, d = w.u (alpha_0 = g_0 / d_0, beta_0 = 0).
// The product A u_{k+1} needs the neighbours' u_{k+1}: each row forms them
// on the fly from the neighbours' r_k, w_k and s_{k-1}, with the very
// operation their owner uses, so r, w and s are double-buffered by iteration
// parity.  One iteration is one launch that begins by summing the partials
// the previous launch left, in the same fixed order in every workgroup, so
// every workgroup holds the same alpha, beta and stopping test without a
// reduction launch, a fence or an atomic; the partials are double-buffered
// by parity too, since a workgroup that finishes early writes its partials
// while a late one may still be summing the previous set.  Once the stopping
// test holds every later launch returns at once, so the host queues many
// iterations between reads of the scalars.
//
// Workspace (doubles): two sets (by parity) of per-row records {r, w, s,
// diag} [2][4 n] (a neighbour's operands are one 32-byte record, not four
// scattered doubles), p [n], block partials of r.u, w.u and r.r
// [2][3][grid] and of b.b [grid], then the scalars (CgScal).
//
// Workgroups of a CG launch: more rows per thread on large trees, but fewer
// partials for every workgroup to sum and fewer workgroups to dispatch
// (avalanche solves: 12.8 us per iteration at 1024, 11.6 at 512, 12.4 at 256).
#ifndef PIC_CG_GRID_MAX
#define PIC_CG_GRID_MAX 512
#endif
static_assert(PIC_CG_GRID_MAX % kBlock == 0 && PIC_CG_GRID_MAX <= 1024, "partials are loaded kBlock at a time");
int cg_grid(uint32_t n) {
  int g = (int)ceil_div(n, kBlock);
  return g < PIC_CG_GRID_MAX ? g : PIC_CG_GRID_MAX;
}
int cg_ws_doubles(uint32_t n) {
  return (int)(9u * n + 7u * (uint32_t)cg_grid(n) + (uint32_t)((sizeof(CgScal) + 7) / 8));
}
size_t cg_scalars_offset(uint32_t n) { return 9u * (size_t)n + 7u * (size_t)cg_grid(n); }

struct __attribute__((aligned(32))) CgRec {
  double r, w, s, d;
};

struct CgView {
  CgRec* rec[2];
  double* p;
  double *pg[2], *pd[2], *prr[2], *pbb;
  CgScal* sc;
};
__device__ __forceinline__ CgView cg_view(double* ws, uint32_t n, int grid) {
  CgView v;
  v.rec[0] = (CgRec*)ws;
  v.rec[1] = (CgRec*)(ws + 4u * (size_t)n);
  v.p = ws + 8u * (size_t)n;
  double* part = ws + 9u * (size_t)n;
  for (int b = 0; b < 2; ++b) {
    v.pg[b] = part + (size_t)(3 * b) * grid;
    v.pd[b] = part + (size_t)(3 * b + 1) * grid;
    v.prr[b] = part + (size_t)(3 * b + 2) * grid;
  }
  v.pbb = part + (size_t)6 * grid;
  v.sc = (CgScal*)(v.pbb + grid);
  return v;
}

// Sum over the workgroup; the result is valid in every thread.
__device__ __forceinline__ double block_sum_all(double v) {
  __shared__ double red[kBlock / 64];
  v = wave_sum(v);
  if (lane_id() == 0) red[threadIdx.x / 64] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) t = t + red[w];
  __syncthreads();
  return t;
}

// Sum of the partials part[0 .. gridDim.x) in a fixed order; every
// workgroup gets the same value, valid in every thread.
__device__ __forceinline__ double sum_partials(const double* part) {
  double a = 0.0;
  for (uint32_t j = threadIdx.x; j < gridDim.x; j += kBlock) a += part[j];
  return block_sum_all(a);
}

// Three workgroup sums in one pass through LDS (one pair of barriers).
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c) {
  __shared__ double red3[3][kBlock / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  if (lane_id() == 0) {
    red3[0][threadIdx.x / 64] = a;
    red3[1][threadIdx.x / 64] = b;
    red3[2][threadIdx.x / 64] = c;
  }
  __syncthreads();
  a = b = c = 0.0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    a = a + red3[0][w];
    b = b + red3[1][w];
    c = c + red3[2][w];
  }
  __syncthreads();
}
// The partials of three arrays summed together, each in the fixed order of
// sum_partials.
__device__ __forceinline__ void sum_partials3(const double* pa, const double* pb, const double* pc, double& a,
                                              double& b, double& c) {
  a = b = c = 0.0;
  for (uint32_t j = threadIdx.x; j < gridDim.x; j += kBlock) {
    a += pa[j];
    b += pb[j];
    c += pc[j];
  }
  block_sum3(a, b, c);
}

// (A v)_i for a vector given row by row through f(j); U neighbours are
// fetched at a time
template <int U = 8, class F>
__device__ __forceinline__ double apply_row(const Stencil2D& st, uint32_t i, double vi, F f) {
  double y = st.diag[i] * vi;
  const uint32_t* nb = st.nbr + (size_t)i * 8u;
  const uint32_t code = st.code[i];
#pragma unroll U
  for (int c = 0; c < 8; ++c) y = y - face_coef((code >> (2 * c)) & 3u) * f(nb[c]);
  return y;
}

// r = b - A x; partials of b.b
__global__ __launch_bounds__(kBlock) void k_cg_setup(Mesh2D m, Stencil2D st, const unsigned long long* __restrict__ Q,
                                                     int nspecies, double k0, double k1, const double* __restrict__ x,
                                                     double* ws) {
  const uint32_t n = m.nleaves;
  const CgView w = cg_view(ws, n, (int)gridDim.x);
  double sbb = 0.0;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    double b = (double)(long long)Q[i] * k0;
    if (nspecies > 1) b = b + (double)(long long)Q[(size_t)n + i] * k1;
    b = b + st.bnd[i];
    const double ax = apply_row(st, i, x[i], [&](uint32_t j) { return x[j]; });
    const double dg = st.diag[i];
    w.rec[0][i].r = b - ax;
    w.rec[0][i].d = dg;
    w.rec[1][i].d = dg;
    sbb += b * b;
  }
  sbb = block_sum_all(sbb);
  if (threadIdx.x == 0) {
    w.pbb[blockIdx.x] = sbb;
    if (blockIdx.x == 0) {
      w.sc->done = 0u;
      w.sc->it = 0u;
    }
  }
}

// u_0 = r_0 / diag, w_0 = A u_0, s_{-1} = p_{-1} = 0; partials of r.u, w.u
// and r.r
__global__ __launch_bounds__(kBlock) void k_cg_start(Mesh2D m, Stencil2D st, double* ws) {
  const uint32_t n = m.nleaves;
  const CgView w = cg_view(ws, n, (int)gridDim.x);
  CgRec* __restrict__ rc = w.rec[0];
  double sg = 0.0, sd = 0.0, srr = 0.0;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double ri = rc[i].r;
    const double ui = ri / rc[i].d;
    const double wi = apply_row(st, i, ui, [&](uint32_t j) { return rc[j].r / rc[j].d; });
    rc[i].w = wi;
    rc[i].s = 0.0;
    w.p[i] = 0.0;
    sg += ri * ui;
    sd += wi * ui;
    srr += ri * ri;
  }
  block_sum3(sg, sd, srr);
  if (threadIdx.x == 0) {
    w.pg[0][blockIdx.x] = sg;
    w.pd[0][blockIdx.x] = sd;
    w.prr[0][blockIdx.x] = srr;
  }
}

// s_k, r_{k+1} and u_{k+1} of one row from its r_k, w_k, s_{k-1}: the same
// operations for the owner and for every neighbour that needs its u_{k+1}
struct CgNext {
  double s, r, u;
};
__device__ __forceinline__ CgNext cg_next(double rk, double wk, double sk1, double dg, double alpha, double beta) {
  CgNext o;
  o.s = fma(beta, sk1, wk);
  o.r = fma(-alpha, o.s, rk);
  o.u = o.r / dg;
  return o;
}

// Operands of one row that do not depend on alpha and beta: its own r_k,
// w_k, s_{k-1}, p_{k-1}, x_k, diagonal and face codes, and its neighbours'
// r_k, w_k, s_{k-1} and diagonals.
struct CgRow {
  double dg, r, w, s, p, x;
  uint32_t code;
  double nr[8], nw[8], ns[8], nd[8];
};
__device__ __forceinline__ void cg_load_row(const Stencil2D& st, const CgRec* __restrict__ rc,
                                            const double* __restrict__ P, const double* __restrict__ x, uint32_t i,
                                            CgRow& a) {
  const CgRec o = rc[i];
  a.dg = o.d;
  a.r = o.r;
  a.w = o.w;
  a.s = o.s;
  a.p = P[i];
  a.x = x[i];
  a.code = st.code[i];
  const uint32_t* nb = st.nbr + (size_t)i * 8u;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const CgRec q = rc[nb[c]];
    a.nr[c] = q.r;
    a.nw[c] = q.w;
    a.ns[c] = q.s;
    a.nd[c] = q.d;
  }
}
// The row's update: s_k, p_k, x_{k+1}, r_{k+1}, u_{k+1} and w_{k+1} = (A u_{k+1})_i
// (the diagonal term first, then the eight neighbours in stencil order).
struct CgOut {
  CgNext o;
  double p, x, w;
};
__device__ __forceinline__ CgOut cg_row(const CgRow& a, double alpha, double beta) {
  CgOut r;
  r.o = cg_next(a.r, a.w, a.s, a.dg, alpha, beta);
  r.p = fma(beta, a.p, a.r / a.dg);
  r.x = fma(alpha, r.p, a.x);
  double y = a.dg * r.o.u;
#pragma unroll
  for (int c = 0; c < 8; ++c)
    y = y - face_coef((a.code >> (2 * c)) & 3u) * cg_next(a.nr[c], a.nw[c], a.ns[c], a.nd[c], alpha, beta).u;
  r.w = y;
  return r;
}

// Iteration k: the stopping test on r_k.r_k (rr <= rtol2 bb, or k = maxit),
// alpha_k and beta_k, then s_k, p_k, x_{k+1}, r_{k+1}, w_{k+1} = A u_{k+1}
// and the partials of r.u, w.u and r.r after the update.  The loads of the
// partials, of the thread's first row and of its neighbours are all issued
// before the partials are reduced: none of them depends on alpha or beta.
constexpr int kCgPartLoads = PIC_CG_GRID_MAX / kBlock;   // cg_grid() <= PIC_CG_GRID_MAX workgroups
__global__ __launch_bounds__(kBlock) void k_cg_iter(Mesh2D m, Stencil2D st, double* __restrict__ x, double* ws,
                                                    uint32_t k, double rtol2, uint32_t maxit) {
  const uint32_t n = m.nleaves;
  const CgView w = cg_view(ws, n, (int)gridDim.x);
  CgScal* S = w.sc;
  const bool odd = (k & 1u) != 0u;   // selects, not an index: keeps the view in registers
  const double* __restrict__ pg = odd ? w.pg[1] : w.pg[0];
  const double* __restrict__ pd = odd ? w.pd[1] : w.pd[0];
  const double* __restrict__ pr = odd ? w.prr[1] : w.prr[0];
  // partials of the previous launch, in the order sum_partials takes them
  double vg[kCgPartLoads], vd[kCgPartLoads], vr[kCgPartLoads];
#pragma unroll
  for (int q = 0; q < kCgPartLoads; ++q) {
    const uint32_t j = threadIdx.x + (uint32_t)q * kBlock;
    const uint32_t jj = j < gridDim.x ? j : 0u;
    vg[q] = pg[jj];
    vd[q] = pd[jj];
    vr[q] = pr[jj];
  }
  const CgRec* __restrict__ rc = odd ? w.rec[1] : w.rec[0];
  const uint32_t i0 = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t stride = gridDim.x * kBlock;
  CgRow a;
  if (i0 < n) cg_load_row(st, rc, w.p, x, i0, a);
  if (S->done) return;   // uniform over the launch (nothing has been written)
  double g = 0.0, d = 0.0, rr = 0.0;
#pragma unroll
  for (int q = 0; q < kCgPartLoads; ++q) {
    if (threadIdx.x + (uint32_t)q * kBlock < gridDim.x) {
      g += vg[q];
      d += vd[q];
      rr += vr[q];
    }
  }
  block_sum3(g, d, rr);
  const double bb = k == 0u ? sum_partials(w.pbb) : S->bb;
  const bool stop = rr <= rtol2 * bb || k >= maxit;
  const double beta = k == 0u ? 0.0 : g / S->gam[(k - 1u) & 1u];
  const double alpha = k == 0u ? g / d : g / (d - beta * g / S->alf[(k - 1u) & 1u]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S->gam[k & 1u] = g;
    S->alf[k & 1u] = alpha;
    S->rr = rr;
    if (k == 0u) S->bb = bb;
    S->it = k;
    if (stop) S->done = 1u;
  }
  if (stop) return;
  CgRec* __restrict__ rn = odd ? w.rec[0] : w.rec[1];
  double sg = 0.0, sd = 0.0, srr = 0.0;
  for (uint32_t i = i0; i < n; i += stride) {
    if (i != i0) cg_load_row(st, rc, w.p, x, i, a);
    const CgOut u = cg_row(a, alpha, beta);
    w.p[i] = u.p;
    x[i] = u.x;
    rn[i].r = u.o.r;   // the record's diagonal stays
    rn[i].w = u.w;
    rn[i].s = u.o.s;
    sg += u.o.r * u.o.u;
    sd += u.w * u.o.u;
    srr += u.o.r * u.o.r;
  }
  block_sum3(sg, sd, srr);
  if (threadIdx.x == 0) {
    (odd ? w.pg[0] : w.pg[1])[blockIdx.x] = sg;
    (odd ? w.pd[0] : w.pd[1])[blockIdx.x] = sd;
    (odd ? w.prr[0] : w.prr[1])[blockIdx.x] = srr;
  }
}

hipError_t launch_cg_setup(const Mesh2D& m, const Stencil2D& st, const unsigned long long* Q, int nspecies,
                           const double* kappa, double* x, double* ws, hipStream_t s) {
  const int g = cg_grid(m.nleaves);
  hipLaunchKernelGGL(k_cg_setup, dim3(g), dim3(kBlock), 0, s, m, st, Q, nspecies, kappa[0], kappa[1], x, ws);
  hipLaunchKernelGGL(k_cg_start, dim3(g), dim3(kBlock), 0, s, m, st, ws);
  return hipGetLastError();
}

hipError_t launch_cg_iter(const Mesh2D& m, const Stencil2D& st, double* x, double* ws, uint32_t k, double rtol2,
                          uint32_t maxit, hipStream_t s) {
  const int g = cg_grid(m.nleaves);
  hipLaunchKernelGGL(k_cg_iter, dim3(g), dim3(kBlock), 0, s, m, st, x, ws, k, rtol2, maxit);
  return hipGetLastError();
}

#define PIC_FIELD_INST(T)                                                                                        \
  template hipError_t launch_field1d<T>(const InstDev<T>*, int, int, int, const double*, hipStream_t);          \
  template hipError_t launch_dipic_field<T>(const InstDev<T>&, hipStream_t);                                   \
  template hipError_t launch_node_e_1d<T>(const InstDev<T>&, const double*, int, hipStream_t);                 \
  template hipError_t launch_corner_field<T>(const Mesh2D&, const double*, double*, double*, T*, hipStream_t);   \
  template hipError_t launch_corner_field3<T>(const Mesh2D&, const double*, double*, double*, T*, hipStream_t);  \
  template hipError_t launch_round_table<T>(const double*, T*, int64_t, hipStream_t);
PIC_FIELD_INST(float)
PIC_FIELD_INST(double)

}  // namespace pic
