// Device-side geometry of the structured trace spaces and the per-face /
// per-macro-element work items shared by the grid kernels (trace.hip) and
// the single-workgroup coarse tail (tail.hip).
#pragma once
#include "hdg_internal.hpp"

namespace hdg {
namespace dev {

// Arithmetic type of the cycle kernels: the vector storage type T.  The
// operator blocks may be stored narrower than the vectors (M = float under
// T = double: the FP32 copies read by the 3D mixed cycle); sums then run in
// the vectors' FP64.  A row of a trace operator applied to a smooth vector
// cancels to a small fraction of its terms' magnitudes: in 3D (k = 3,
// tau = 1) a cycle with FP32 vectors or FP32 sums loses the digits the coarse
// correction needs and stalls CG near a relative residual of 1e-6, while FP32
// operator blocks under FP64 vectors and sums keep the FP64 cycle's
// iteration count.  In 2D the FP32 cycle keeps CG within 1% of the FP64
// count.
template <typename T>
struct AccOf {
  using type = T;
};
template <typename T>
using acc_t = typename AccOf<T>::type;

// one lane's entry group (vw<T>() values) of an AoSoA operator block
template <typename T>
__device__ inline void ld_group(const T* p, T* out) {
  constexpr int V = vw<T>();
  if constexpr (V == 1) {
    out[0] = p[0];
  } else {
    typedef T vt __attribute__((ext_vector_type(V)));
    const vt v = *reinterpret_cast<const vt*>(p);
#pragma unroll
    for (int q = 0; q < V; ++q) out[q] = v[q];
  }
}

// acc += (stored block) * x for the CNT entries of one AoSoA item starting at
// blk (= base + aos_item).  Entry e pairs output o and input i as
// (o, i) = (e % NMINOR, e / NMINOR) when OUT_MINOR, else (e / NMINOR, e % NMINOR).
// Every output accumulates in increasing input order.
template <typename T, int CNT, int NMINOR, bool OUT_MINOR, typename X, typename Y>
__device__ inline void aos_mv(const T* __restrict__ blk, const X* x, Y* acc) {
  constexpr int V = vw<T>();
  constexpr int NG = (CNT + V - 1) / V;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    T v[V];
    ld_group<T>(blk + g * (LANES * V), v);
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const int e = g * V + q;
      if (e < CNT) {
        if (OUT_MINOR)
          acc[e % NMINOR] += Y(v[q]) * x[e / NMINOR];
        else
          acc[e / NMINOR] += Y(v[q]) * x[e % NMINOR];
      }
    }
  }
}

// acc[e % NE] += blk[B + e] * x[e / NE] for e in [0, NE * NE): one slot's
// NE x NE block of a face matrix (entries B .. B + NE*NE - 1 of the item).
// Groups that straddle two slots are loaded by both (the second load hits
// the cache), so each slot can sit in its own branch.
template <typename T, int NE, typename X, typename Y>
__device__ inline void aos_mv_slot(const T* __restrict__ blk, int B, const X* x, Y* acc) {
  constexpr int V = vw<T>();
  const int g0 = B / V, g1 = (B + NE * NE - 1) / V;
#pragma unroll
  for (int g = g0; g <= g1; ++g) {
    T v[V];
    ld_group<T>(blk + g * (LANES * V), v);
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const int e = g * V + q - B;
      if (e >= 0 && e < NE * NE) acc[e % NE] += Y(v[q]) * x[e / NE];
    }
  }
}

template <int D>
__device__ inline long nface_dir(int n) {
  long v = n - 1;
  for (int a = 1; a < D; ++a) v *= n;
  return v;
}

// interior face id of normal c at grid coordinates g (g[c] in 1..n-1)
template <int D>
__device__ inline long face_id(int c, const int* g, int n) {
  long idx = 0, stride = 1;
  for (int a = 0; a < D; ++a) {
    if (a == c) {
      idx += (long)(g[a] - 1) * stride;
      stride *= (n - 1);
    } else {
      idx += (long)g[a] * stride;
      stride *= n;
    }
  }
  return c * nface_dir<D>(n) + idx;
}

// 32-bit index arithmetic: face and element counts stay below 2^31 for every
// supported mesh (n <= 8192 in 2D, 512 in 3D)
template <int D>
__device__ inline int decode_face(long F, int n, int* g) {
  const unsigned nfd = (unsigned)nface_dir<D>(n);
  const unsigned f = (unsigned)F;
  const int c = (int)(f / nfd);
  unsigned r = f - (unsigned)c * nfd;
  for (int a = 0; a < D; ++a) {
    const unsigned ext = a == c ? (unsigned)(n - 1) : (unsigned)n;
    const unsigned q = r / ext;
    g[a] = (int)(r - q * ext) + (a == c ? 1 : 0);
    r = q;
  }
  return c;
}

template <int D>
__device__ inline void decode_elem(long T, int n, int* e) {
  unsigned t = (unsigned)T;
  for (int a = 0; a < D; ++a) {
    const unsigned q = t / (unsigned)n;
    e[a] = (int)(t - q * (unsigned)n);
    t = q;
  }
}

template <int D>
__device__ inline long elem_id(const int* e, int n) {
  long T = 0;
  for (int a = D - 1; a >= 0; --a) T = T * n + e[a];
  return T;
}

// length of the trace vector of a level with n^D elements and ne values per
// face (interior faces only); several right-hand sides are stored one after
// another with this stride
template <int D>
__device__ inline long trace_len(int n, int ne) {
  return (long)D * nface_dir<D>(n) * ne;
}

// p + k, or null when p is null
template <typename P>
__device__ inline P off(P p, long k) {
  return p ? p + k : p;
}

// XCD-aware face blocks.  Workgroups are dealt to the 8 XCDs round-robin
// (workgroup p runs on XCD p % 8), and each XCD has its own L2.  The faces of
// each normal direction are cut into 8 contiguous chunks of C blocks of 256;
// XCD j takes chunk j of every direction, i.e. the same band of grid rows in
// every direction, so the neighbouring traces a face gathers were mostly
// fetched into the same L2 (with the plain mapping every XCD touches almost
// every line of the vector).  Returns the face of lane tid of workgroup p, or
// -1 for the padding lanes.  The matching grid has 8 * D * C workgroups.
template <int D>
__device__ inline long xcd_face(int n, unsigned p, unsigned tid) {
  const unsigned nfd = (unsigned)nface_dir<D>(n);
  const unsigned C = ((nfd + 255u) / 256u + 7u) / 8u;
  const unsigned j = p & 7u, m = p >> 3;
  const unsigned c = m / C, w = m - c * C;
  const unsigned local = (j * C + w) * 256u + tid;
  if (c >= (unsigned)D || local >= nfd) return -1;
  return (long)c * nfd + local;
}

// Several right-hand sides: the right-hand side index runs fastest after the
// XCD, so the nrhs workgroups that read the same operator chunk are dealt to
// the same XCD back to back and share it through its L2.  Also returns the
// right-hand side and a reduction slot laid out [rhs][8 * D * C].
template <int D>
__device__ inline long xcd_face_rhs(int n, int nrhs, unsigned p, unsigned tid, int* rhs, unsigned* slot) {
  const unsigned nfd = (unsigned)nface_dir<D>(n);
  const unsigned C = ((nfd + 255u) / 256u + 7u) / 8u;
  const unsigned j = p & 7u, m = p >> 3;
  const unsigned r = m % (unsigned)nrhs, m2 = m / (unsigned)nrhs;
  *rhs = (int)r;
  *slot = r * (8u * D * C) + j + 8u * m2;
  const unsigned c = m2 / C, w = m2 - c * C;
  const unsigned local = (j * C + w) * 256u + tid;
  if (c >= (unsigned)D || local >= nfd) return -1;
  return (long)c * nfd + local;
}

// interior faces of a coarse macro-element m (grid n/2) on the fine grid n:
// iota = c * 2^(D-1) + lex(t) over the tangential child bits t.
template <int D>
__device__ inline long macro_iface(const int* m, int iota, int n) {
  constexpr int NS = 1 << (D - 1);
  const int c = iota / NS, t = iota % NS;
  int g[3] = {0, 0, 0};
  int j = 0;
  for (int a = 0; a < D; ++a) {
    if (a == c) {
      g[a] = 2 * m[a] + 1;
    } else {
      g[a] = 2 * m[a] + ((t >> j) & 1);
      ++j;
    }
  }
  return face_id<D>(c, g, n);
}

// weight of coarse vertex V at fine vertex v of sub-face t of a macro-face
template <int D>
__device__ inline double jh_weight(int t, int v, int V) {
  double w = 1.0;
#pragma unroll
  for (int j = 0; j < D - 1; ++j) {
    double s = 0.5 * (((t >> j) & 1) + ((v >> j) & 1));
    w *= ((V >> j) & 1) ? s : 1.0 - s;
  }
  return w;
}

// sub-face t of coarse face with grid coords G (coarse grid) on the fine grid
template <int D>
__device__ inline long subface(int c, const int* G, int t, int n) {
  int g[3] = {0, 0, 0};
  int j = 0;
  for (int a = 0; a < D; ++a) {
    if (a == c) {
      g[a] = 2 * G[a];
    } else {
      g[a] = 2 * G[a] + ((t >> j) & 1);
      ++j;
    }
  }
  return face_id<D>(c, g, n);
}

// ---------------------------------------------------------------------------
// Fused h-transition kernels (2D).  A macro-element M of the coarse grid owns
// its NIF interior faces (I) exclusively and sees its NBF boundary sub-faces
// (B) from its own children only; every output is written by one lane.
//   I face iota = c*NS + t (t: tangential child bit), sides = children with
//   bit c = 0 / 1;  B face beta = (2c+sd)*NS + t, the child inside M is on
//   face-major side 1-sd.
// Child ch, local slot (cc, sd2) lies on M-face: q = bit_cc(ch) + sd2;
//   q == 1 -> I face cc*NS + t(ch, cc); else B face (2cc + (q==2))*NS + t.
template <int D>
struct Macro {
  static constexpr int NC = 1 << (D - 1);
  static constexpr int NS = NC;
  static constexpr int NIF = D * NS;
  static constexpr int NBF = 2 * D * NS;
  static constexpr int NL = 2 * D * NC;
  static constexpr int NI = NIF * NC;
  static constexpr int NCL = 2 * D * NC;
};

template <int D>
__device__ inline int tbits(int ch, int cc) {
  int t = 0, j = 0;
  for (int a = 0; a < D; ++a)
    if (a != cc) {
      t |= ((ch >> a) & 1) << j;
      ++j;
    }
  return t;
}

// M-face index (0..NIF-1 interior, NIF.. boundary) of child ch's slot sl
template <int D>
__device__ inline int mface_of(int ch, int sl) {
  constexpr int NS = 1 << (D - 1);
  const int cc = sl / 2, sd2 = sl % 2;
  const int q = ((ch >> cc) & 1) + sd2;
  const int t = tbits<D>(ch, cc);
  if (q == 1) return cc * NS + t;
  return D * NS + (2 * cc + (q == 2 ? 1 : 0)) * NS + t;
}

// fine face id of M-face mf (-1 on the domain boundary), and for B faces the
// face-major side holding M's child
template <int D>
__device__ inline long mface_id(const int* m, int mf, int n, int* side_in) {
  constexpr int NS = 1 << (D - 1);
  constexpr int NIF = D * NS;
  int g[3] = {0, 0, 0};
  int c, t;
  if (mf < NIF) {
    c = mf / NS;
    t = mf % NS;
    g[c] = 2 * m[c] + 1;
    *side_in = -1;
  } else {
    const int b = mf - NIF;
    const int S = b / NS;
    t = b % NS;
    c = S / 2;
    const int sd = S % 2;
    g[c] = 2 * m[c] + 2 * sd;
    *side_in = 1 - sd;
    if (g[c] == 0 || g[c] == n) return -1;
  }
  int j = 0;
  for (int a = 0; a < D; ++a)
    if (a != c) {
      g[a] = 2 * m[a] + ((t >> j) & 1);
      ++j;
    }
  return face_id<D>(c, g, n);
}

// (A e) on face fid, side `side` only (child ch), e given per M-face
template <int D, typename T>
__device__ inline void side_apply(const T* __restrict__ Af, long fid, int side, int ch,
                                  const acc_t<T> (*eM)[1 << (D - 1)], acc_t<T>* acc) {
  using Mc = Macro<D>;
  constexpr int NE = Mc::NC, NL = Mc::NL;
  constexpr long S = vpad<T>(NL * NE);
  const T* Mb = Af + aos_item<T>(fid, 2 * S) + side * S * LANES;
  acc_t<T> xs[NL];
#pragma unroll
  for (int sl = 0; sl < 2 * D; ++sl) {
    const int mf = mface_of<D>(ch, sl);
#pragma unroll
    for (int bb = 0; bb < NE; ++bb) xs[sl * NE + bb] = eM[mf][bb];
  }
  aos_mv<T, NL * NE, NE, true>(Mb, xs, acc);
}

// child of M on side `side` of I face iota
template <int D>
__device__ inline int ichild(int iota, int side) {
  constexpr int NS = 1 << (D - 1);
  const int c = iota / NS, t = iota % NS;
  int ch = side << c, j = 0;
  for (int a = 0; a < D; ++a)
    if (a != c) {
      ch |= ((t >> j) & 1) << a;
      ++j;
    }
  return ch;
}

template <int D>
__device__ inline int bchild(int b) {  // b = beta - NIF
  constexpr int NS = 1 << (D - 1);
  const int S = b / NS, t = b % NS;
  const int c = S / 2, sd = S % 2;
  int ch = sd << c, j = 0;
  for (int a = 0; a < D; ++a)
    if (a != c) {
      ch |= ((t >> j) & 1) << a;
      ++j;
    }
  return ch;
}

// x[i NC + a] for face i >= 0, else 0.  The load is issued in either case
// (from face 0 when i < 0) and the value selected afterwards.  In the
// multi-lane transition items and the one-lane prolongation a load under a
// condition was waited for before the next one was issued, so the faces of
// a macro-element were fetched one round trip after another.  (The one-lane
// pre-coarse item keeps its conditional loads: there they were not
// serialized, and issuing all of them at once measured slower.)
template <int NC, typename T>
__device__ inline acc_t<T> face_val_or0(const T* x, long i, int a) {
  const T v = x[(i >= 0 ? i : 0) * NC + a];
  return i >= 0 ? acc_t<T>(v) : acc_t<T>(0);
}

// Pre-coarse-correction work of level l for one macro-element:
//   rho_I = r_I - (A e)_I, e_I += A_II^-1 rho_I (if do_corr),
//   cb_M = -J^T (A_M e)_B + P_M^T rho_I      (its share of Q (r - A e))
template <int D, typename T>
__device__ inline void hpre_item(long M, int n, const T* __restrict__ Af, const T* __restrict__ AIIinv,
                                 const T* __restrict__ P, const T* r, T* e, int do_corr, T* cb) {
  using Mc = Macro<D>;
  using A = acc_t<T>;
  constexpr int NC = Mc::NC, NIF = Mc::NIF, NBF = Mc::NBF, NI = Mc::NI, NCL = Mc::NCL, NS = Mc::NS;
  const int nm = n / 2;
  int m[3] = {0, 0, 0};
  decode_elem<D>(M, nm, m);
  A eM[NIF + NBF][NC];
  long fid[NIF + NBF];
  int sidein[NIF + NBF];
#pragma unroll
  for (int f = 0; f < NIF + NBF; ++f) {
    fid[f] = mface_id<D>(m, f, n, &sidein[f]);
#pragma unroll
    for (int a = 0; a < NC; ++a) eM[f][a] = fid[f] >= 0 ? A(e[fid[f] * NC + a]) : A(0);
  }
  A rho[NI];
#pragma unroll
  for (int i = 0; i < NIF; ++i) {
    A acc[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) acc[a] = A(0);
    side_apply<D, T>(Af, fid[i], 0, ichild<D>(i, 0), eM, acc);
    side_apply<D, T>(Af, fid[i], 1, ichild<D>(i, 1), eM, acc);
#pragma unroll
    for (int a = 0; a < NC; ++a) rho[i * NC + a] = A(r[fid[i] * NC + a]) - acc[a];
  }
  if (do_corr) {
    A s[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) s[i] = A(0);
    aos_mv<T, NI * NI, NI, false>(AIIinv + aos_item<T>(M, vpad<T>(NI * NI)), rho, s);
#pragma unroll
    for (int i = 0; i < NIF; ++i)
#pragma unroll
      for (int a = 0; a < NC; ++a) e[fid[i] * NC + a] = T(eM[i][a] + s[i * NC + a]);
  }
  A out[NCL];
#pragma unroll
  for (int j = 0; j < NCL; ++j) out[j] = A(0);
  aos_mv<T, NI * NCL, NCL, true>(P + aos_item<T>(M, vpad<T>(NI * NCL)), rho, out);
#pragma unroll
  for (int b = 0; b < NBF; ++b) {
    const int f = NIF + b;
    if (fid[f] < 0) continue;
    A acc[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) acc[a] = A(0);
    side_apply<D, T>(Af, fid[f], sidein[f], bchild<D>(b), eM, acc);
    const int S = b / NS, t = b % NS;
#pragma unroll
    for (int V = 0; V < NC; ++V) {
      A s = A(0);
#pragma unroll
      for (int v = 0; v < NC; ++v) s += A(jh_weight<D>(t, v, V)) * acc[v];
      out[S * NC + V] -= s;
    }
  }
#pragma unroll
  for (int j = 0; j < NCL; ++j) cb[M * NCL + j] = T(out[j]);
}

// The same pre-coarse work spread over L = 2 or 4 lanes of one wavefront per
// macro-element (2D): lane q owns interior faces q QF .. q QF + QF - 1
// (QF = 4 / L) and the boundary faces of macro-faces q QS .. q QS + QS - 1
// (QS = 4 / L), whose restriction shares are exactly the coarse DOFs of
// those macro-faces.  The interior residual is exchanged with shuffles; each
// lane then forms its rows of A_II^-1 rho and its columns of P^T rho.  The
// serial chain of loads per lane shrinks about L-fold, which is what bounds
// latency-bound levels.  All L lanes of a group are active together (the
// group's macro-element is in range or not).
template <typename T, int L>
__device__ inline void hpreL_item(long M, int q, int n, const T* __restrict__ Af, const T* __restrict__ AIIinv,
                                  const T* __restrict__ P, const T* r, T* e, int do_corr, T* cb) {
  static_assert(L == 2 || L == 4, "2 or 4 lanes per macro-element");
  using Mc = Macro<2>;
  using A = acc_t<T>;
  constexpr int NC = Mc::NC, NS = Mc::NS, NIF = Mc::NIF, NBF = Mc::NBF, NI = Mc::NI, NCL = Mc::NCL;
  constexpr int QF = NIF / L, QS = 4 / L;
  const int base = (int)(threadIdx.x & 63) & ~(L - 1);
  const int nm = n / 2;
  int m[3] = {0, 0, 0};
  decode_elem<2>(M, nm, m);
  A eM[NIF + NBF][NC];
  long fid[NIF + NBF];
  int sidein[NIF + NBF];
#pragma unroll
  for (int f = 0; f < NIF + NBF; ++f) {
    fid[f] = mface_id<2>(m, f, n, &sidein[f]);
#pragma unroll
    for (int a = 0; a < NC; ++a) eM[f][a] = face_val_or0<NC, T>(e, fid[f], a);
  }
  A rq[QF][NC];
#pragma unroll
  for (int u = 0; u < QF; ++u) {
    const int i = q * QF + u;
    A acc[NC] = {A(0), A(0)};
    side_apply<2, T>(Af, fid[i], 0, ichild<2>(i, 0), eM, acc);
    side_apply<2, T>(Af, fid[i], 1, ichild<2>(i, 1), eM, acc);
#pragma unroll
    for (int a = 0; a < NC; ++a) rq[u][a] = A(r[fid[i] * NC + a]) - acc[a];
  }
  A rho[NI];
#pragma unroll
  for (int src = 0; src < L; ++src)
#pragma unroll
    for (int u = 0; u < QF; ++u)
#pragma unroll
      for (int a = 0; a < NC; ++a) rho[(src * QF + u) * NC + a] = __shfl(rq[u][a], base + src, 64);
  if (do_corr) {
#pragma unroll
    for (int u = 0; u < QF; ++u) {
      const int i = q * QF + u;
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        const int row = i * NC + a;
        A sacc = A(0);
#pragma unroll
        for (int j = 0; j < NI; ++j) sacc += A(AIIinv[aos_off<T>(M, vpad<T>(NI * NI), row * NI + j)]) * rho[j];
        e[fid[i] * NC + a] = T(eM[i][a] + sacc);
      }
    }
  }
#pragma unroll
  for (int w = 0; w < QS; ++w) {
    const int S = q * QS + w;
    A o[NC];
#pragma unroll
    for (int V = 0; V < NC; ++V) {
      A sacc = A(0);
#pragma unroll
      for (int i = 0; i < NI; ++i) sacc += A(P[aos_off<T>(M, vpad<T>(NI * NCL), i * NCL + S * NC + V)]) * rho[i];
      o[V] = sacc;
    }
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int b = S * NS + t;
      const int f = NIF + b;
      // no such face on the domain boundary: formed from face 0's block
      // (loads issued with the others) and dropped
      const bool has = fid[f] >= 0;
      A ab[NC] = {A(0), A(0)};
      side_apply<2, T>(Af, has ? fid[f] : 0, sidein[f], bchild<2>(b), eM, ab);
#pragma unroll
      for (int V = 0; V < NC; ++V) {
        A sacc = A(0);
#pragma unroll
        for (int v = 0; v < NC; ++v) sacc += A(jh_weight<2>(t, v, V)) * ab[v];
        if (has) o[V] -= sacc;
      }
    }
#pragma unroll
    for (int V = 0; V < NC; ++V) cb[M * NCL + S * NC + V] = T(o[V]);
  }
}

// Coarse residual r_c = J^T r_B + cb_{M-} + cb_{M+} per coarse face, and the
// first block-Jacobi step of the coarse level e_c = D^-1 r_c (when Dc given)
template <int D, typename T>
__device__ inline void hsum_item(long Fc, int n, const T* r, const T* cb, const T* __restrict__ Dc, T* rc, T* ec) {
  constexpr int NC = 1 << (D - 1);
  using A = acc_t<T>;
  constexpr int NCL = 2 * D * NC;
  const int nm = n / 2;
  int G[3] = {0, 0, 0};
  const int c = decode_face<D>(Fc, nm, G);
  A out[NC];
#pragma unroll
  for (int V = 0; V < NC; ++V) out[V] = A(0);
#pragma unroll
  for (int t = 0; t < NC; ++t) {
    const long f = subface<D>(c, G, t, n);
#pragma unroll
    for (int v = 0; v < NC; ++v) {
      const A rv = r[f * NC + v];
#pragma unroll
      for (int V = 0; V < NC; ++V) out[V] += A(jh_weight<D>(t, v, V)) * rv;
    }
  }
  int mm[3] = {G[0], G[1], G[2]};
  mm[c] = G[c] - 1;
  const long Mm = elem_id<D>(mm, nm);
  mm[c] = G[c];
  const long Mp = elem_id<D>(mm, nm);
#pragma unroll
  for (int V = 0; V < NC; ++V) {
    out[V] += A(cb[Mm * NCL + (2 * c + 1) * NC + V]);
    out[V] += A(cb[Mp * NCL + (2 * c) * NC + V]);
    rc[Fc * NC + V] = T(out[V]);
  }
  if (Dc) {
    A s[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) s[a] = A(0);
    aos_mv<T, NC * NC, NC, false>(Dc + aos_item<T>(Fc, vpad<T>(NC * NC)), out, s);
#pragma unroll
    for (int a = 0; a < NC; ++a) ec[Fc * NC + a] = T(s[a]);
  }
}

// Out-of-place prolongation and post-correction local correction:
//   e_new = e_old + I e_c (I = [P_M e_c ; J e_c], eq. n_1_Ik), then on I
//   faces e_new_I += A_II^-1 (r - A e_new)_I when do_corr.
// Blocks [0, nbm): one lane per macro-element writes its I faces; blocks
// [nbm, ...): one lane per coarse face writes its B sub-faces.
template <int D, typename T>
__device__ inline void hpost_m_item(long M, int n, const T* __restrict__ Af, const T* __restrict__ AIIinv,
                                    const T* __restrict__ P, const T* r, const T* ec, const T* eold, T* enew,
                                    int do_corr) {
  using Mc = Macro<D>;
  using A = acc_t<T>;
  constexpr int NC = Mc::NC, NIF = Mc::NIF, NBF = Mc::NBF, NI = Mc::NI, NCL = Mc::NCL, NS = Mc::NS;
  const int nm = n / 2;
  {
    int m[3] = {0, 0, 0};
    decode_elem<D>(M, nm, m);
    A cv[NCL];
#pragma unroll
    for (int sl = 0; sl < 2 * D; ++sl) {
      const int cc = sl / 2, sd = sl % 2;
      const int p = m[cc] + sd;
      // coarse face on the domain boundary: no value (zero); its load reads
      // the face at position 1 and is dropped, so no load waits on a branch
      const bool in = !(p == 0 || p == nm);
      int G[3] = {m[0], m[1], m[2]};
      G[cc] = in ? p : 1;
      const long Fc = face_id<D>(cc, G, nm);
#pragma unroll
      for (int V = 0; V < NC; ++V) {
        const T v = ec[Fc * NC + V];
        cv[sl * NC + V] = in ? A(v) : A(0);
      }
    }
    A eM[NIF + NBF][NC];
    long fid[NIF + NBF];
    int sidein[NIF + NBF];
#pragma unroll
    for (int f = 0; f < NIF + NBF; ++f) {
      fid[f] = mface_id<D>(m, f, n, &sidein[f]);
#pragma unroll
      for (int a = 0; a < NC; ++a) eM[f][a] = face_val_or0<NC, T>(eold, fid[f], a);
    }
    // B faces: e + J e_c (local copy only; the coarse-face lanes write them)
#pragma unroll
    for (int b = 0; b < NBF; ++b) {
      const int f = NIF + b;
      if (fid[f] < 0) continue;
      const int S = b / NS, t = b % NS;
#pragma unroll
      for (int v = 0; v < NC; ++v) {
        A s = A(0);
#pragma unroll
        for (int V = 0; V < NC; ++V) s += A(jh_weight<D>(t, v, V)) * cv[S * NC + V];
        eM[f][v] += s;
      }
    }
    {
      A s[NI];
#pragma unroll
      for (int i = 0; i < NI; ++i) s[i] = A(0);
      aos_mv<T, NI * NCL, NCL, false>(P + aos_item<T>(M, vpad<T>(NI * NCL)), cv, s);
#pragma unroll
      for (int i = 0; i < NIF; ++i)
#pragma unroll
        for (int a = 0; a < NC; ++a) eM[i][a] += s[i * NC + a];
    }
    if (do_corr) {
      A rho[NI];
#pragma unroll
      for (int i = 0; i < NIF; ++i) {
        A acc[NC];
#pragma unroll
        for (int a = 0; a < NC; ++a) acc[a] = A(0);
        side_apply<D, T>(Af, fid[i], 0, ichild<D>(i, 0), eM, acc);
        side_apply<D, T>(Af, fid[i], 1, ichild<D>(i, 1), eM, acc);
#pragma unroll
        for (int a = 0; a < NC; ++a) rho[i * NC + a] = A(r[fid[i] * NC + a]) - acc[a];
      }
      A s[NI];
#pragma unroll
      for (int i = 0; i < NI; ++i) s[i] = A(0);
      aos_mv<T, NI * NI, NI, false>(AIIinv + aos_item<T>(M, vpad<T>(NI * NI)), rho, s);
#pragma unroll
      for (int i = 0; i < NIF; ++i)
#pragma unroll
        for (int a = 0; a < NC; ++a) enew[fid[i] * NC + a] = T(eM[i][a] + s[i * NC + a]);
    } else {
#pragma unroll
      for (int i = 0; i < NIF; ++i)
#pragma unroll
        for (int a = 0; a < NC; ++a) enew[fid[i] * NC + a] = T(eM[i][a]);
    }
  }
}

// hpost_m_item over L = 2 or 4 lanes per macro-element (2D), as hpreL_item:
// lane q prolongs onto its interior faces, the prolonged interior values and
// then the interior residual are exchanged with shuffles, and lane q applies
// its rows of A_II^-1.
template <typename T, int L>
__device__ inline void hpostL_m_item(long M, int q, int n, const T* __restrict__ Af, const T* __restrict__ AIIinv,
                                     const T* __restrict__ P, const T* r, const T* ec, const T* eold, T* enew,
                                     int do_corr) {
  static_assert(L == 2 || L == 4, "2 or 4 lanes per macro-element");
  using Mc = Macro<2>;
  using A = acc_t<T>;
  constexpr int NC = Mc::NC, NIF = Mc::NIF, NBF = Mc::NBF, NI = Mc::NI, NCL = Mc::NCL, NS = Mc::NS;
  constexpr int QF = NIF / L;
  const int base = (int)(threadIdx.x & 63) & ~(L - 1);
  const int nm = n / 2;
  int m[3] = {0, 0, 0};
  decode_elem<2>(M, nm, m);
  A cv[NCL];
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    const int cc = sl / 2, sd = sl % 2;
    const int p = m[cc] + sd;
    const bool in = !(p == 0 || p == nm);  // boundary: load face 1's value, select zero
    int G[3] = {m[0], m[1], m[2]};
    G[cc] = in ? p : 1;
    const long Fc = face_id<2>(cc, G, nm);
#pragma unroll
    for (int V = 0; V < NC; ++V) {
      const T v = ec[Fc * NC + V];
      cv[sl * NC + V] = in ? A(v) : A(0);
    }
  }
  A eM[NIF + NBF][NC];
  long fid[NIF + NBF];
  int sidein[NIF + NBF];
#pragma unroll
  for (int f = 0; f < NIF + NBF; ++f) {
    fid[f] = mface_id<2>(m, f, n, &sidein[f]);
#pragma unroll
    for (int a = 0; a < NC; ++a) eM[f][a] = face_val_or0<NC, T>(eold, fid[f], a);
  }
  // B faces: e + J e_c (local copies only)
#pragma unroll
  for (int b = 0; b < NBF; ++b) {
    const int f = NIF + b;
    if (fid[f] < 0) continue;
    const int S = b / NS, t = b % NS;
#pragma unroll
    for (int v = 0; v < NC; ++v) {
      A sacc = A(0);
#pragma unroll
      for (int V = 0; V < NC; ++V) sacc += A(jh_weight<2>(t, v, V)) * cv[S * NC + V];
      eM[f][v] += sacc;
    }
  }
  // own interior faces: e + P e_c, then shared
  A eq[QF][NC];
#pragma unroll
  for (int u = 0; u < QF; ++u) {
    const int i = q * QF + u;
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      A sacc = A(0);
#pragma unroll
      for (int j = 0; j < NCL; ++j) sacc += A(P[aos_off<T>(M, vpad<T>(NI * NCL), (i * NC + a) * NCL + j)]) * cv[j];
      eq[u][a] = eM[i][a] + sacc;
    }
  }
#pragma unroll
  for (int src = 0; src < L; ++src)
#pragma unroll
    for (int u = 0; u < QF; ++u)
#pragma unroll
      for (int a = 0; a < NC; ++a) eM[src * QF + u][a] = __shfl(eq[u][a], base + src, 64);
  if (!do_corr) {
#pragma unroll
    for (int u = 0; u < QF; ++u)
#pragma unroll
      for (int a = 0; a < NC; ++a) enew[fid[q * QF + u] * NC + a] = T(eq[u][a]);
    return;
  }
  A rq[QF][NC];
#pragma unroll
  for (int u = 0; u < QF; ++u) {
    const int i = q * QF + u;
    A acc[NC] = {A(0), A(0)};
    side_apply<2, T>(Af, fid[i], 0, ichild<2>(i, 0), eM, acc);
    side_apply<2, T>(Af, fid[i], 1, ichild<2>(i, 1), eM, acc);
#pragma unroll
    for (int a = 0; a < NC; ++a) rq[u][a] = A(r[fid[i] * NC + a]) - acc[a];
  }
  A rho[NI];
#pragma unroll
  for (int src = 0; src < L; ++src)
#pragma unroll
    for (int u = 0; u < QF; ++u)
#pragma unroll
      for (int a = 0; a < NC; ++a) rho[(src * QF + u) * NC + a] = __shfl(rq[u][a], base + src, 64);
#pragma unroll
  for (int u = 0; u < QF; ++u) {
    const int i = q * QF + u;
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      A sacc = A(0);
#pragma unroll
      for (int j = 0; j < NI; ++j) sacc += A(AIIinv[aos_off<T>(M, vpad<T>(NI * NI), (i * NC + a) * NI + j)]) * rho[j];
      enew[fid[i] * NC + a] = T(eq[u][a] + sacc);
    }
  }
}

template <int D, typename T>
__device__ inline void hpost_f_item(long Fc, int n, const T* ec, const T* eold, T* enew) {
  constexpr int NC = 1 << (D - 1);
  using A = acc_t<T>;
  const int nm = n / 2;
  {
    int G[3] = {0, 0, 0};
    const int c = decode_face<D>(Fc, nm, G);
    A cv[NC];
#pragma unroll
    for (int V = 0; V < NC; ++V) cv[V] = ec[Fc * NC + V];
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const long f = subface<D>(c, G, t, n);
#pragma unroll
      for (int v = 0; v < NC; ++v) {
        A s = eold[f * NC + v];
#pragma unroll
        for (int V = 0; V < NC; ++V) s += A(jh_weight<D>(t, v, V)) * cv[V];
        enew[f * NC + v] = T(s);
      }
    }
  }
}


// acc = (A x)_F for interior face F: both element matrices touching F, read
// from the face-major AoSoA form (stored as M; vectors as T).  Returns the
// face's normal direction.
template <int D, int NE, typename T, typename M = T>
__device__ inline int face_acc(long F, int n, const M* __restrict__ Af, const T* x, acc_t<T>* acc) {
  constexpr int NL = 2 * D * NE;
  constexpr long S = vpad<M>(NL * NE);
  int g[3] = {0, 0, 0};
  const int c = decode_face<D>(F, n, g);
#pragma unroll
  for (int a = 0; a < NE; ++a) acc[a] = acc_t<T>(0);
  const M* Mbase = Af + aos_item<M>(F, 2 * S);
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    int e[3] = {g[0], g[1], g[2]};
    e[c] = g[c] - 1 + side;
    const M* Mx = Mbase + side * S * LANES;
#pragma unroll
    for (int sl = 0; sl < 2 * D; ++sl) {
      const int cc = sl / 2, sd = sl % 2;
      const int p = e[cc] + sd;
      if constexpr (NE <= 2) {
        // P1 face blocks (the coarse levels, latency-bound): every slot's
        // loads go out together.  A boundary slot reads the face at
        // position 1 and its update is dropped by the select; a load under
        // the branch was waited for before the next slot's.
        const bool in = !(p == 0 || p == n);
        int fg[3] = {e[0], e[1], e[2]};
        fg[cc] = in ? p : 1;
        const T* xf = x + face_id<D>(cc, fg, n) * NE;
        acc_t<T> xs[NE], t[NE];
#pragma unroll
        for (int bb = 0; bb < NE; ++bb) {
          xs[bb] = xf[bb];
          t[bb] = acc[bb];
        }
        aos_mv_slot<M, NE>(Mx, sl * NE * NE, xs, t);
#pragma unroll
        for (int bb = 0; bb < NE; ++bb) acc[bb] = in ? t[bb] : acc[bb];
      } else {
        // a boundary slot carries no unknowns; the branch also keeps the
        // compiler from hoisting the loads of every slot at once (registers)
        if (p == 0 || p == n) continue;
        int fg[3] = {e[0], e[1], e[2]};
        fg[cc] = p;
        const T* xf = x + face_id<D>(cc, fg, n) * NE;
        acc_t<T> xs[NE];
#pragma unroll
        for (int bb = 0; bb < NE; ++bb) xs[bb] = xf[bb];
        aos_mv_slot<M, NE>(Mx, sl * NE * NE, xs, acc);
      }
    }
  }
  return c;
}

// Blocks of 256 items for several right-hand sides on the XCDs: workgroup p
// of a grid of xcd_rhs_grid(nb, nrhs) takes block b of right-hand side rhs.
// XCD p % 8 holds the contiguous blocks [j C, (j + 1) C) of every right-hand
// side, and the right-hand side runs fastest after the XCD, so the
// workgroups that read one block's operator data run on one XCD back to back
// and share it through its L2.  Returns -1 for padding workgroups.  With one
// right-hand side the grid is the nb blocks in plain order (measured faster
// there).
__device__ inline long xcd_block_rhs(long nb, int nrhs, unsigned p, int* rhs) {
  if (nrhs == 1) {
    *rhs = 0;
    return (long)p < nb ? (long)p : -1;
  }
  const unsigned C = (unsigned)((nb + 7) / 8);
  const unsigned j = p & 7u, m = p >> 3;
  *rhs = (int)(m % (unsigned)nrhs);
  const unsigned w = m / (unsigned)nrhs;
  const long b = (long)j * C + w;
  return (w < C && b < nb) ? b : -1;
}

// Element-major XCD-aware blocks (same idea as xcd_face over the n^D
// elements, in bands of whole grid rows): element of lane tid of workgroup p
// and its right-hand side, or -1 for padding lanes.  Grid 8 * C * nrhs.
__device__ inline long xcd_elem_rhs(long nelem, int nrhs, unsigned p, unsigned tid, int* rhs) {
  const unsigned C = (unsigned)(((nelem + 255) / 256 + 7) / 8);
  const unsigned j = p & 7u, m = p >> 3;
  const unsigned r = m % (unsigned)nrhs, w = m / (unsigned)nrhs;
  *rhs = (int)r;
  const long T = ((long)j * C + w) * 256 + tid;
  return (w < C && T < nelem) ? T : -1;
}

// offset of entry i of element T in an element-major AoSoA array of `per`
// entries per element
__device__ inline long elem_aos(long T, int per, int i) { return (T >> 6) * (long)per * LANES + (long)i * LANES + (T & 63); }

// acc = A^e x_T for element T from the packed upper triangle: gather the
// element's traces (zero on the boundary), then one pass over the triangle,
// each entry feeding both a_ij x_j into row i and a_ij x_i into row j.
template <int D, int NE, typename T>
__device__ inline void elem_prod(long Tq, int n, const T* __restrict__ Ap, const T* x, acc_t<T>* acc) {
  using A = acc_t<T>;
  constexpr int NL = 2 * D * NE, NPK = NL * (NL + 1) / 2;
  int e[3] = {0, 0, 0};
  decode_elem<D>(Tq, n, e);
  A xs[NL];
#pragma unroll
  for (int sl = 0; sl < 2 * D; ++sl) {
    const int cc = sl / 2, sd = sl % 2;
    const int p = e[cc] + sd;
    if (p == 0 || p == n) {
#pragma unroll
      for (int b = 0; b < NE; ++b) xs[sl * NE + b] = A(0);
    } else {
      int fg[3] = {e[0], e[1], e[2]};
      fg[cc] = p;
      const T* xf = x + face_id<D>(cc, fg, n) * NE;
#pragma unroll
      for (int b = 0; b < NE; ++b) xs[sl * NE + b] = xf[b];
    }
  }
#pragma unroll
  for (int i = 0; i < NL; ++i) acc[i] = A(0);
  constexpr int W = pvw<T>();
  const T* ap = Ap + pk_off<T>(Tq, NPK, 0);
  int idx = 0;
  T v[W];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
#pragma unroll
    for (int j = i; j < NL; ++j, ++idx) {
      if (idx % W == 0) {
        if constexpr (W == 1) {
          v[0] = ap[(long)idx * LANES];
        } else {
          typedef T vt __attribute__((ext_vector_type(W)));
          const vt g = *reinterpret_cast<const vt*>(ap + (long)(idx / W) * (LANES * W));
#pragma unroll
          for (int q = 0; q < W; ++q) v[q] = g[q];
        }
      }
      const A a = v[idx % W];
      acc[i] += a * xs[j];
      if (j != i) acc[j] += a * xs[i];
    }
  }
}

// z_T = A^e x_T stored element-major (first phase of the two-phase apply)
template <int D, int NE, typename T>
__device__ inline void elem_item(long Tq, int n, const T* __restrict__ Ap, const T* x, T* z) {
  constexpr int NL = 2 * D * NE;
  acc_t<T> acc[NL];
  elem_prod<D, NE, T>(Tq, n, Ap, x, acc);
  T* zp = z + elem_aos(Tq, NL, 0);
#pragma unroll
  for (int i = 0; i < NL; ++i) zp[(long)i * LANES] = T(acc[i]);
}

// second phase: (A x)_F = z_{T-}[slot 2c+1 rows] + z_{T+}[slot 2c rows]
template <int D, int NE, typename T>
__device__ inline int face_acc_z(long F, int n, const T* z, acc_t<T>* acc) {
  constexpr int NL = 2 * D * NE;
  int g[3] = {0, 0, 0};
  const int c = decode_face<D>(F, n, g);
  int em[3] = {g[0], g[1], g[2]};
  em[c] = g[c] - 1;
  const T* zm = z + elem_aos(elem_id<D>(em, n), NL, (2 * c + 1) * NE);
  const T* zq = z + elem_aos(elem_id<D>(g, n), NL, 2 * c * NE);
#pragma unroll
  for (int a = 0; a < NE; ++a) acc[a] = acc_t<T>(zm[(long)a * LANES]) + acc_t<T>(zq[(long)a * LANES]);
  return c;
}

// y = x + Dinv_F res (one block-Jacobi update of face F; x == nullptr: 0);
// the blocks stored as M, vectors as T
template <int NE, typename T, typename M = T>
__device__ inline void dinv_update(long F, const M* __restrict__ Dinv, const T* x, const acc_t<T>* res, T* y) {
  acc_t<T> s[NE];
#pragma unroll
  for (int a = 0; a < NE; ++a) s[a] = x ? acc_t<T>(x[F * NE + a]) : acc_t<T>(0);
  aos_mv<M, NE * NE, NE, false>(Dinv + aos_item<M>(F, vpad<M>(NE * NE)), res, s);
#pragma unroll
  for (int a = 0; a < NE; ++a) y[F * NE + a] = T(s[a]);
}

// as dinv_update with the block stored as its upper triangle, row by row
// (the symmetric inverse of an SPD block; element-major levels)
template <int NE, typename T>
__device__ inline void dinv_update_sym(long F, const T* __restrict__ Dinv, const T* x, const acc_t<T>* res, T* y) {
  using A = acc_t<T>;
  constexpr int NP = NE * (NE + 1) / 2, V = vw<T>();
  A s[NE];
#pragma unroll
  for (int a = 0; a < NE; ++a) s[a] = x ? A(x[F * NE + a]) : A(0);
  const T* blk = Dinv + aos_item<T>(F, vpad<T>(NP));
  int idx = 0;
  T v[V];
#pragma unroll
  for (int i = 0; i < NE; ++i) {
#pragma unroll
    for (int j = i; j < NE; ++j, ++idx) {
      if (idx % V == 0) ld_group<T>(blk + (idx / V) * (LANES * V), v);
      const A d = A(v[idx % V]);
      s[i] += d * res[j];
      if (j != i) s[j] += d * res[i];
    }
  }
#pragma unroll
  for (int a = 0; a < NE; ++a) y[F * NE + a] = T(s[a]);
}

// one block-Jacobi sweep / residual / apply for interior face F
template <int D, int NE, typename T, int MODE>
__device__ inline void face_item(long F, int n, const T* __restrict__ Af, const T* __restrict__ Dinv, const T* x,
                                 const T* b, T* y) {
  using A = acc_t<T>;
  A acc[NE];
  face_acc<D, NE, T>(F, n, Af, x, acc);
  if (MODE == APPLY_SWEEP) {
    A res[NE];
#pragma unroll
    for (int a = 0; a < NE; ++a) res[a] = A(b[F * NE + a]) - acc[a];
    dinv_update<NE, T>(F, Dinv, x, res, y);
  } else if (MODE == APPLY_RES) {
#pragma unroll
    for (int a = 0; a < NE; ++a) y[F * NE + a] = T(A(b[F * NE + a]) - acc[a]);
  } else {
#pragma unroll
    for (int a = 0; a < NE; ++a) y[F * NE + a] = T(acc[a]);
  }
}

// Output of one face given acc = (A x)_F, per mode (x, b, y, rc, y32
// already offset to the face's right-hand side); reductions add to part.
// DSYM: the level's face-block inverses are stored as upper triangles.  M:
// storage type of the face-block inverses (T, or FP32 under FP64 vectors).
template <int D, int NE, typename T, int MODE, bool DSYM = false, typename M = T>
__device__ inline void face_finish(long F, const acc_t<T>* acc, const M* __restrict__ Dinv, const T* x,
                                   const T* __restrict__ bvec, T* __restrict__ y, const double* __restrict__ Jp,
                                   T* __restrict__ rc, float* __restrict__ y32, double& part) {
  constexpr int NC = 1 << (D - 1);
  using A = acc_t<T>;
  if (MODE == APPLY_Y) {
#pragma unroll
    for (int a = 0; a < NE; ++a) y[F * NE + a] = T(acc[a]);
  } else if (MODE == APPLY_RES) {
#pragma unroll
    for (int a = 0; a < NE; ++a) y[F * NE + a] = T(A(bvec[F * NE + a]) - acc[a]);
  } else if (MODE == APPLY_SWEEP || MODE == APPLY_SWEEP_DOT) {
    A res[NE];
#pragma unroll
    for (int a = 0; a < NE; ++a) res[a] = A(bvec[F * NE + a]) - acc[a];
    if constexpr (DSYM)
      dinv_update_sym<NE, T>(F, Dinv, x, res, y);
    else
      dinv_update<NE, T, M>(F, Dinv, x, res, y);
    if (MODE == APPLY_SWEEP_DOT)  // Jp holds the FP64 vector of the dot product
#pragma unroll
      for (int a = 0; a < NE; ++a) part += Jp[F * NE + a] * (double)y[F * NE + a];
  } else if (MODE == APPLY_RES_PRESTRICT) {  // residual restricted by J_N^T (p-coarsening)
    A res[NE];
#pragma unroll
    for (int a = 0; a < NE; ++a) res[a] = A(bvec[F * NE + a]) - acc[a];
    A rcv[NC];
#pragma unroll
    for (int v = 0; v < NC; ++v) {
      A s = A(0);
#pragma unroll
      for (int a = 0; a < NE; ++a) s += A(Jp[a * NC + v]) * res[a];
      rc[F * NC + v] = T(s);
      rcv[v] = A(T(s));  // the coarse first step starts from the stored residual
    }
    if (y)  // first block-Jacobi step of the P1 level: y = D_c^-1 rc (Dinv = coarse blocks)
      dinv_update<NC, T, M>(F, Dinv, (const T*)nullptr, rcv, y);
  } else if (MODE == APPLY_Y_DOT) {
#pragma unroll
    for (int a = 0; a < NE; ++a) {
      y[F * NE + a] = T(acc[a]);
      part += (double)x[F * NE + a] * (double)T(acc[a]);
    }
  } else {  // APPLY_RES_NORM
#pragma unroll
    for (int a = 0; a < NE; ++a) {
      const T v = T(A(bvec[F * NE + a]) - acc[a]);
      y[F * NE + a] = v;
      if (y32) y32[F * NE + a] = (float)v;
      part += (double)v * (double)v;
    }
  }
}

template <int NE, typename T, bool DSYM = false, typename M = T>
__device__ inline void jacobi0_item(long F, const M* __restrict__ Dinv, const T* r, T* e) {
  acc_t<T> rv[NE];
#pragma unroll
  for (int b = 0; b < NE; ++b) rv[b] = r[F * NE + b];
  if constexpr (DSYM)
    dinv_update_sym<NE, T>(F, Dinv, (const T*)nullptr, rv, e);
  else
    dinv_update<NE, T, M>(F, Dinv, (const T*)nullptr, rv, e);
}


}  // namespace dev
}  // namespace hdg
