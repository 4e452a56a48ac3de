// Forward kernels of the selective Fock-amplitude sweep (gfx950).
//
// One sweep step S handles every lattice point m with |m| = S of the detected
// box.  At m it applies, in this order (Algorithm 1, Sec. 3.1.3; Algorithm 2,
// Sec. 3.2, where every node is a block of undetected-mode entries):
//   * the diagonal pivot d(m) (needed when b != 0 or modes are undetected):
//     it writes the type-1 offsets d(m) + 1_i at weight 2S+1, reading its own
//     value (the b term of Eq. recrel, and the undetected neighbours of the
//     block) and the type-1 offsets of the previous step;
//   * the off-diagonal / bridge pivots d(m) + 1_ket(K) for K up to the first
//     non-zero mode of m: they write F0(m + 1_K), F2(K)(m), F1010(K,.)(m) and
//     F1001(K,.)(m) at weight 2S+2 from the previous step's even families.
// Every target is written by exactly one pivot (its canonical parent), so the
// kernels are pure gathers with no atomics.  All targets of one step are
// independent (Sec. 2.2, the two parallelisations), which gives one launch per
// step.
#include <algorithm>
#include <cstring>

#include "fd_device.h"

namespace fd {

// ---------------------------------------------------------------------------
// prep: caller's triple (block order) -> interleaved internal positions,
// A symmetrised; input finiteness and the b = 0 promise checked on device.
// ---------------------------------------------------------------------------
struct PrepArgs {
  int pos2blk[kMaxPos];
  int npos, M2, check_b_zero;
};

template <typename R>
__global__ void k_prep(const cx<R>* __restrict__ A, const cx<R>* __restrict__ b, const cx<R>* __restrict__ c,
                       cx<R>* __restrict__ Ai, cx<R>* __restrict__ bi, cx<R>* __restrict__ ci,
                       cx<R>* __restrict__ f0node0, PrepArgs a, int* status) {
  const int npos = a.npos, M2 = a.M2;
  int bad = 0;
  for (int idx = threadIdx.x; idx < npos * npos; idx += blockDim.x) {
    const int p = idx / npos, q = idx % npos;
    const int pb = a.pos2blk[p], qb = a.pos2blk[q];
    const cx<R> u = ld(A + (size_t)pb * M2 + qb), v = ld(A + (size_t)qb * M2 + pb);
    const cx<R> s = cmake<R>(R(0.5) * (u.x + v.x), R(0.5) * (u.y + v.y));
    if (!isfinite(s.x) || !isfinite(s.y)) bad |= 1;
    st(Ai + idx, s);
  }
  for (int p = threadIdx.x; p < npos; p += blockDim.x) st(bi + p, ld(b + a.pos2blk[p]));
  for (int p = threadIdx.x; p < M2; p += blockDim.x) {
    const cx<R> v = ld(b + p);
    if (!isfinite(v.x) || !isfinite(v.y)) bad |= 1;
    if (a.check_b_zero && (v.x != R(0) || v.y != R(0))) bad |= 2;
  }
  if (threadIdx.x == 0) {
    const cx<R> cv = ld(c);
    if (!isfinite(cv.x) || !isfinite(cv.y)) bad |= 1;
    st(ci, cv);
    if (f0node0) st(f0node0, cv);  // G_0 = c (Sec. 2.2 vacuum amplitude)
  }
  if (bad) atomicOr(status, bad);
}

// ---------------------------------------------------------------------------
// Step 1 of Algorithm 2: the whole undetected block at zero detections.
// Entry kappa != 0 is pulled from its parent kappa - 1_q, q = first non-zero
// coordinate, by Eq. recrel restricted to the undetected positions.  One
// wavefront, the block in LDS, entries visited by weight (host-built list).
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(64) void k_ufill(DevPlan P, const cx<R>* __restrict__ Ai,
                                              const cx<R>* __restrict__ bi, cx<R>* G,
                                              const int* __restrict__ elist, const int* __restrict__ woff,
                                              int wmax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<R>* g = reinterpret_cast<cx<R>*>(smem_raw);
  const int nq = P.nq, npos = P.npos, B = P.B;
  const int lane = threadIdx.x;
  if (lane == 0) g[0] = ld(G);   // c, written by the prep kernel
  wave_sync();
  for (int w = 1; w <= wmax; ++w) {
    for (int t = woff[w] + lane; t < woff[w + 1]; t += 64) {
      const int e = elist[t];
      int kap[kMaxUq];
      int rem = e;
#pragma unroll
      for (int q = 0; q < kMaxUq; ++q) {
        kap[q] = q < nq ? rem / P.ustride[q] : 0;
        rem -= kap[q] * (q < nq ? P.ustride[q] : 0);
      }
      int qf = nq;
#pragma unroll
      for (int q = kMaxUq - 1; q >= 0; --q)
        if (q < nq && kap[q] > 0) qf = q;
      const int pe = e - P.ustride[qf];
      cx<R> acc = czero<R>();
      cfma(acc, ld(bi + qf), g[pe]);
#pragma unroll
      for (int q = 0; q < kMaxUq; ++q) {
        if (q >= nq) continue;
        const int pq = kap[q] - (q == qf ? 1 : 0);
        if (pq > 0) cfma(acc, ld(Ai + qf * npos + q), cscale(g[pe - P.ustride[q]], sqrt(R(pq))));
      }
      g[e] = cscale(acc, R(1) / sqrt(R(kap[qf])));
    }
    wave_sync();
  }
  for (int e = lane; e < B; e += 64) st(G + e, g[e]);
}

// ---------------------------------------------------------------------------
// Shared-memory prologue: PN table and sqrt tables.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void load_tables(const DevPlan& P, int* spn, R* sq, R* isq) {
  const int n = (P.MD + 1) * P.pnw;
  for (int i = threadIdx.x; i < n; i += blockDim.x) spn[i] = P.pn[i];
  for (int v = threadIdx.x; v < kMaxCut + 4; v += blockDim.x) {
    sq[v] = sqrt(R(v));
    isq[v] = v ? R(1) / sqrt(R(v)) : R(0);
  }
}

// ---------------------------------------------------------------------------
// Algorithm 1 (every mode detected): one thread per lattice point.
// ---------------------------------------------------------------------------
template <int MD, bool ODD, typename R>
__global__ __launch_bounds__(kThreads) void k_fwd_point(DevPlan P, LevelPtrs<R> L, const cx<R>* __restrict__ Ai,
                                                        const cx<R>* __restrict__ bi, int S, int nwork) {
  constexpr int NP = 2 * MD;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* sq = reinterpret_cast<R*>(smem_raw);
  R* isq = sq + (kMaxCut + 4);
  int* spn = reinterpret_cast<int*>(isq + (kMaxCut + 4));
  load_tables(P, spn, sq, isq);
  __syncthreads();
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nwork) return;
  const int pnw = P.pnw;
  int m[MD], s[MD + 1], rdn[MD], rup[MD];
  unrank<MD>(spn, pnw, P.CD, S, r, m, s);
  neighbour_ranks<MD>(spn, pnw, s, rdn, rup);

  const cx<R> g0 = ld(L.f0cur + r);
  cx<R> yk[MD];
#pragma unroll
  for (int K = 0; K < MD; ++K) yk[K] = czero<R>();

  if (ODD && m[0] <= P.CD[0] - 2) {
    // diagonal pivot d(m): reads d(m) - 1_l, writes d(m) + 1_i (type-1 offsets)
    cx<R> x[NP];
#pragma unroll
    for (int j = 0; j < MD; ++j) {
      if (m[j] > 0) {
        x[2 * j] = cscale(ld(L.rd[fam_f1b(MD, j)] + rdn[j]), sq[m[j]]);   // d(m)-1_ket(j) = F1b(j)(m-1_j)
        x[2 * j + 1] = cscale(ld(L.rd[fam_f1k(j)] + rdn[j]), sq[m[j]]);   // d(m)-1_bra(j) = F1k(j)(m-1_j)
      } else {
        x[2 * j] = czero<R>();
        x[2 * j + 1] = czero<R>();
      }
    }
#pragma unroll
    for (int j = 0; j < MD; ++j) {
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int i = 2 * j + side;
        cx<R> acc = czero<R>();
        cfma(acc, ld(bi + i), g0);
#pragma unroll
        for (int l = 0; l < NP; ++l) cfma(acc, ld(Ai + i * NP + l), x[l]);
        acc = cscale(acc, isq[m[j] + 1]);
        if (side == 0) {
          yk[j] = acc;
          if (j == 0 || m[j] <= P.CD[j] - 2) st(L.wr[fam_f1k(j)] + r, acc);
        } else {
          const bool ok = (j == 0) ? (m[0] <= P.CD[0] - 3) : (m[j] <= P.CD[j] - 2);
          if (ok) st(L.wr[fam_f1b(MD, j)] + r, acc);
        }
      }
    }
  }

  int K0 = MD;
#pragma unroll
  for (int d = MD - 1; d >= 0; --d)
    if (m[d] > 0) K0 = d;
#pragma unroll
  for (int K = 0; K < MD; ++K) {
    if (K > K0) break;
    if (m[K] > P.CD[K] - 2) continue;
    // pivot p = d(m) + 1_ket(K): reads p - 1_l for l >= ket(K)
    cx<R> x[NP];
    x[2 * K] = cscale(g0, sq[m[K] + 1]);                                    // p - 1_ket(K) = d(m)
    x[2 * K + 1] = (m[K] > 0) ? cscale(ld(L.rd[fam_f2(MD, K)] + rdn[K]), sq[m[K]]) : czero<R>();
#pragma unroll
    for (int j = K + 1; j < MD; ++j) {
      if (m[j] > 0) {
        x[2 * j] = cscale(ld(L.rd[fam_1001(MD, K, j)] + rdn[j]), sq[m[j]]);
        x[2 * j + 1] = cscale(ld(L.rd[fam_1010(MD, K, j)] + rdn[j]), sq[m[j]]);
      } else {
        x[2 * j] = czero<R>();
        x[2 * j + 1] = czero<R>();
      }
    }
    // writes p + 1_i
#pragma unroll
    for (int i = 2 * K; i < NP; ++i) {
      const int j = i >> 1;
      bool ok;
      R scale;
      cx<R>* dst;
      if (i == 2 * K + 1) {                 // d(m + 1_K): output amplitude
        ok = true;
        scale = isq[m[K] + 1];
        dst = L.f0nxt + rup[K];
      } else if (i == 2 * K) {              // F2(K)(m)
        ok = (m[K] <= P.CD[K] - 3);
        scale = isq[m[K] + 2];
        dst = L.wr[fam_f2(MD, K)] + r;
      } else {                              // F1010(K,j)(m) / F1001(K,j)(m)
        ok = (m[j] <= P.CD[j] - 2);
        scale = isq[m[j] + 1];
        dst = L.wr[(i & 1) ? fam_1001(MD, K, j) : fam_1010(MD, K, j)] + r;
      }
      if (!ok) continue;
      cx<R> acc = czero<R>();
      if (ODD) cfma(acc, ld(bi + i), yk[K]);
#pragma unroll
      for (int l = 2 * K; l < NP; ++l) cfma(acc, ld(Ai + i * NP + l), x[l]);
      st(dst, cscale(acc, scale));
    }
  }
}

// ---------------------------------------------------------------------------
// Algorithm 2 (undetected modes present).  A node's block of B entries is
// split into chunks of whole rows of the first undetected coordinate (rows of
// R0 = B / C0 entries); one workgroup handles one (lattice point, chunk).
// The pivot's undetected neighbours reach one row back, so a chunk computes
// the pivot rows it needs one row above its own (recomputed, not stored).
// LDS: F0(m) rows [k0-2, k1) and the bridge pivot blocks F1k(K)(m), rows
// [k0-1, k1), for every bridge K applied at m.
// ---------------------------------------------------------------------------
template <int MD, int NQ, typename R>
__global__ __launch_bounds__(kBT) void k_fwd_block(DevPlan P, LevelPtrs<R> L, const cx<R>* __restrict__ Ai,
                                                        const cx<R>* __restrict__ bi, int S, int nwork,
                                                        ChunkGeo G) {
  constexpr int NPD = 2 * MD;
  constexpr int NPOS = NQ + NPD;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int B = P.B, R0 = G.R0;
  cx<R>* lf0 = reinterpret_cast<cx<R>*>(smem_raw);             // (RC + 2) rows
  cx<R>* lpk = lf0 + (size_t)(G.RC + 2) * R0;                  // MD x (RC + 1) rows
  cx<R>* sA = lpk + (size_t)MD * (G.RC + 1) * R0;      // A (NPOS x NPOS) then b (NPOS)
  const cx<R>* sb = sA + NPOS * NPOS;
  R* sq = reinterpret_cast<R*>(sA + NPOS * NPOS + NPOS);
  R* isq = sq + (kMaxCut + 4);
  int* spn = reinterpret_cast<int*>(isq + (kMaxCut + 4));
  load_tables(P, spn, sq, isq);
  for (int i = threadIdx.x; i < NPOS * NPOS + NPOS; i += blockDim.x) sA[i] = ld(Ai + i);
  __syncthreads();
  const int pnw = P.pnw;
  const int pk1 = (G.RC + 1) * R0;   // entries of one pivot block in LDS
  for (int w = blockIdx.x; w < nwork * G.nchunks; w += gridDim.x) {
    const int r = w / G.nchunks, c = w - r * G.nchunks;
    const int k0 = c * G.RC, k1 = min(G.C0, k0 + G.RC);
    int m[MD], s[MD + 1], rdn[MD], rup[MD];
    unrank<MD>(spn, pnw, P.CD, S, r, m, s);
    neighbour_ranks<MD>(spn, pnw, s, rdn, rup);
    int K0 = MD;
#pragma unroll
    for (int d = MD - 1; d >= 0; --d)
      if (m[d] > 0) K0 = d;
    if (m[0] > P.CD[0] - 2) continue;   // no pivot at this point (uniform)
    const size_t rB = (size_t)r * B;
    // F0(m), rows [k0-2, k1)
    {
      const int e0 = max(0, k0 - 2) * R0, e1 = k1 * R0;
      const int base = (k0 - 2) * R0;
      for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) lf0[e - base] = ld(L.f0cur + rB + e);
    }
    __syncthreads();
    // diagonal pivot, rows [k0-1, k1): own rows store every type-1 target,
    // the halo row only keeps the bridge pivot blocks
    {
      const int e0 = max(0, k0 - 1) * R0, e1 = k1 * R0;
      for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const bool own = e >= k0 * R0;
        int kap[NQ];
        int rem = e;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          kap[q] = rem / P.ustride[q];
          rem -= kap[q] * P.ustride[q];
        }
        const int le = e - (k0 - 2) * R0;
        const cx<R> piv = lf0[le];
        cx<R> un[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) un[q] = kap[q] > 0 ? cscale(lf0[le - P.ustride[q]], sq[kap[q]]) : czero<R>();
        cx<R> x[NPD];
#pragma unroll
        for (int j = 0; j < MD; ++j) {
          if (m[j] > 0) {
            x[2 * j] = cscale(ld(L.rd[fam_f1b(MD, j)] + (size_t)rdn[j] * B + e), sq[m[j]]);
            x[2 * j + 1] = cscale(ld(L.rd[fam_f1k(j)] + (size_t)rdn[j] * B + e), sq[m[j]]);
          } else {
            x[2 * j] = czero<R>();
            x[2 * j + 1] = czero<R>();
          }
        }
#pragma unroll
        for (int j = 0; j < MD; ++j) {
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            const int i = 2 * j + side;
            const bool ok = side == 0 ? (j == 0 || m[j] <= P.CD[j] - 2)
                                      : ((j == 0) ? (m[0] <= P.CD[0] - 3) : (m[j] <= P.CD[j] - 2));
            const bool bridge = side == 0 && j <= K0 && m[j] <= P.CD[j] - 2;
            if (!(ok && own) && !bridge) continue;
            const int row = (NQ + i) * NPOS;
            cx<R> acc = czero<R>();
            cfma(acc, sb[NQ + i], piv);
#pragma unroll
            for (int q = 0; q < NQ; ++q) cfma(acc, sA[row + q], un[q]);
#pragma unroll
            for (int l = 0; l < NPD; ++l) cfma(acc, sA[row + NQ + l], x[l]);
            acc = cscale(acc, isq[m[j] + 1]);
            if (ok && own) st(L.wr[side ? fam_f1b(MD, j) : fam_f1k(j)] + rB + e, acc);
            if (bridge) lpk[(size_t)j * pk1 + (e - (k0 - 1) * R0)] = acc;
          }
        }
      }
    }
    __syncthreads();
    // bridges d(m) + 1_ket(K), own rows
#pragma unroll
    for (int K = 0; K < MD; ++K) {
      if (K > K0 || m[K] > P.CD[K] - 2) continue;   // uniform
      const cx<R>* pv = lpk + (size_t)K * pk1;
      for (int e = k0 * R0 + threadIdx.x; e < k1 * R0; e += blockDim.x) {
        int kap[NQ];
        int rem = e;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          kap[q] = rem / P.ustride[q];
          rem -= kap[q] * P.ustride[q];
        }
        const int lp = e - (k0 - 1) * R0;
        const cx<R> piv = pv[lp];
        cx<R> un[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) un[q] = kap[q] > 0 ? cscale(pv[lp - P.ustride[q]], sq[kap[q]]) : czero<R>();
        cx<R> x[NPD];
        x[2 * K] = cscale(lf0[e - (k0 - 2) * R0], sq[m[K] + 1]);
        x[2 * K + 1] = (m[K] > 0) ? cscale(ld(L.rd[fam_f2(MD, K)] + (size_t)rdn[K] * B + e), sq[m[K]]) : czero<R>();
#pragma unroll
        for (int j = K + 1; j < MD; ++j) {
          if (m[j] > 0) {
            x[2 * j] = cscale(ld(L.rd[fam_1001(MD, K, j)] + (size_t)rdn[j] * B + e), sq[m[j]]);
            x[2 * j + 1] = cscale(ld(L.rd[fam_1010(MD, K, j)] + (size_t)rdn[j] * B + e), sq[m[j]]);
          } else {
            x[2 * j] = czero<R>();
            x[2 * j + 1] = czero<R>();
          }
        }
#pragma unroll
        for (int i = 2 * K; i < NPD; ++i) {
          const int j = i >> 1;
          bool ok;
          R scale;
          cx<R>* dst;
          if (i == 2 * K + 1) {
            ok = true;
            scale = isq[m[K] + 1];
            dst = L.f0nxt + (size_t)rup[K] * B + e;
          } else if (i == 2 * K) {
            ok = (m[K] <= P.CD[K] - 3);
            scale = isq[m[K] + 2];
            dst = L.wr[fam_f2(MD, K)] + rB + e;
          } else {
            ok = (m[j] <= P.CD[j] - 2);
            scale = isq[m[j] + 1];
            dst = L.wr[(i & 1) ? fam_1001(MD, K, j) : fam_1010(MD, K, j)] + rB + e;
          }
          if (!ok) continue;
          const int row = (NQ + i) * NPOS;
          cx<R> acc = czero<R>();
          cfma(acc, sb[NQ + i], piv);
#pragma unroll
          for (int q = 0; q < NQ; ++q) cfma(acc, sA[row + q], un[q]);
#pragma unroll
          for (int l = 2 * K; l < NPD; ++l) cfma(acc, sA[row + NQ + l], x[l]);
          st(dst, cscale(acc, scale));
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// F0 (level-major nodes of B entries) -> rho, C order [kappa][n_D].
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kThreads) void k_out_perm(DevPlan P, const cx<R>* __restrict__ f0,
                                                       cx<R>* __restrict__ rho, int64_t N, int64_t total,
                                                       int* status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int* spn = reinterpret_cast<int*>(smem_raw);
  int64_t* slv = reinterpret_cast<int64_t*>(smem_raw + 16 * ((((P.MD + 1) * P.pnw) * 4 + 15) / 16));
  const int npn = (P.MD + 1) * P.pnw;
  for (int i = threadIdx.x; i < npn; i += blockDim.x) spn[i] = P.pn[i];
  for (int i = threadIdx.x; i <= P.smax; i += blockDim.x) slv[i] = P.MD > 0 ? P.lvl[i] : 0;
  __syncthreads();
  const int MD = P.MD, B = P.B, pnw = P.pnw;
  int bad = 0;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t kap = idx / N;
    int64_t rem = idx - kap * N;
    int n[kMaxD];
    int S = 0;
    for (int d = MD - 1; d >= 0; --d) {
      n[d] = (int)(rem % P.CD[d]);
      rem /= P.CD[d];
      S += n[d];
    }
    int rank = 0, sd = S;
    for (int d = 0; d < MD; ++d) {
      rank += pnv(spn, pnw, d + 1, sd) - pnv(spn, pnw, d + 1, sd - n[d]);
      sd -= n[d];
    }
    const cx<R> v = ld(f0 + (size_t)(slv[S] + rank) * B + kap);
    if (!isfinite(v.x) || !isfinite(v.y)) bad = 1;
    st(rho + idx, v);
  }
  if (bad) atomicOr(status, 1);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
// Rows of the first undetected coordinate per chunk: about one wavefront of
// own entries, spread evenly over the rows.
static ChunkGeo chunk_geo(const Plan& Pl) {
  ChunkGeo G;
  G.C0 = Pl.udims[0];
  G.R0 = Pl.B / G.C0;
  int rc = std::max(1, (kBT + G.R0 / 2) / G.R0);
  rc = std::min(rc, G.C0);
  G.nchunks = (G.C0 + rc - 1) / rc;
  G.RC = (G.C0 + G.nchunks - 1) / G.nchunks;
  return G;
}

template <typename R>
static hipError_t launch_fwd_level_t(const Plan& Pl, const DevPlan& P, bool odd, int S, const LevelPtrs<R>& L,
                                     const void* Ai, const void* bi, hipStream_t st) {
  const int MD = Pl.MD;
  if (MD == 0) return hipSuccess;
  const int nwork = (int)Pl.ncnt[S];   // lattice points of level S
  if (nwork <= 0) return hipSuccess;
  const cx<R>* A = reinterpret_cast<const cx<R>*>(Ai);
  const cx<R>* b = reinterpret_cast<const cx<R>*>(bi);
  const size_t tab = 2 * (kMaxCut + 4) * sizeof(R) + (size_t)(MD + 1) * (Pl.smax + 3) * sizeof(int);
  if (Pl.B == 1) {
    const int grid = (nwork + kThreads - 1) / kThreads;
#define FD_LAUNCH_POINT(MDV)                                                                              \
  case MDV:                                                                                               \
    if (odd)                                                                                              \
      hipLaunchKernelGGL((k_fwd_point<MDV, true, R>), dim3(grid), dim3(kThreads), tab, st, P, L, A, b, S, \
                         nwork);                                                                          \
    else                                                                                                  \
      hipLaunchKernelGGL((k_fwd_point<MDV, false, R>), dim3(grid), dim3(kThreads), tab, st, P, L, A, b, \
                         S, nwork);                                                                       \
    break;
    switch (MD) {
      FD_LAUNCH_POINT(1)
      FD_LAUNCH_POINT(2)
      FD_LAUNCH_POINT(3)
      FD_LAUNCH_POINT(4)
      FD_LAUNCH_POINT(5)
      FD_LAUNCH_POINT(6)
      FD_LAUNCH_POINT(7)
      FD_LAUNCH_POINT(8)
      default:
        return hipErrorInvalidValue;
    }
#undef FD_LAUNCH_POINT
  } else {
    const ChunkGeo G = chunk_geo(Pl);
    const size_t shm = (((size_t)(G.RC + 2) + (size_t)MD * (G.RC + 1)) * G.R0 + (size_t)Pl.npos * (Pl.npos + 1)) *
                           sizeof(cx<R>) + tab;
    const int grid = nwork * G.nchunks;
#define FD_LAUNCH_BLOCK(MDV)                                                                               \
  case MDV:                                                                                                \
    if (Pl.nq == 2) {                                                                                      \
      if (shm > 65536)                                                                                     \
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fwd_block<MDV, 2, R>),                 \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);                   \
      hipLaunchKernelGGL((k_fwd_block<MDV, 2, R>), dim3(grid), dim3(kBT), shm, st, P, L, A, b, S,         \
                         nwork, G);                                                                        \
    } else {                                                                                               \
      if (shm > 65536)                                                                                     \
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fwd_block<MDV, 4, R>),                 \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);                   \
      hipLaunchKernelGGL((k_fwd_block<MDV, 4, R>), dim3(grid), dim3(kBT), shm, st, P, L, A, b, S,         \
                         nwork, G);                                                                        \
    }                                                                                                      \
    break;
    switch (MD) {
      FD_LAUNCH_BLOCK(1)
      FD_LAUNCH_BLOCK(2)
      FD_LAUNCH_BLOCK(3)
      FD_LAUNCH_BLOCK(4)
      FD_LAUNCH_BLOCK(5)
      FD_LAUNCH_BLOCK(6)
      FD_LAUNCH_BLOCK(7)
      FD_LAUNCH_BLOCK(8)
      default:
        return hipErrorInvalidValue;
    }
#undef FD_LAUNCH_BLOCK
  }
  return hipGetLastError();
}

// Node-0 pointer of family f of group g at level S.
template <typename R>
static cx<R>* fam_level_ptr(const Plan& Pl, char* base, size_t off, int g, int S, bool ring) {
  if (S < 0) return nullptr;
  const size_t eb = sizeof(cx<R>);
  size_t node = ring ? (size_t)(S & 1) * Pl.maxN[g] : (size_t)Pl.lvl[(size_t)g * (Pl.smax + 2) + S];
  return reinterpret_cast<cx<R>*>(base + off + node * Pl.B * eb);
}

hipError_t launch_prep(const Plan& Pl, const void* A, const void* b, const void* c, void* Ai, void* f0node0,
                       hipStream_t st) {
  PrepArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  for (int p = 0; p < Pl.npos; ++p) pa.pos2blk[p] = Pl.pos2blk[p];
  pa.npos = Pl.npos;
  pa.M2 = 2 * Pl.M;
  pa.check_b_zero = (Pl.flags == FD_B_ZERO) ? 1 : 0;
  const size_t n2 = (size_t)Pl.npos * Pl.npos;
  if (Pl.dt == FD_C64) {
    cx<float>* a = reinterpret_cast<cx<float>*>(Ai);
    hipLaunchKernelGGL((k_prep<float>), dim3(1), dim3(kThreads), 0, st, reinterpret_cast<const cx<float>*>(A),
                       reinterpret_cast<const cx<float>*>(b), reinterpret_cast<const cx<float>*>(c), a, a + n2,
                       a + n2 + Pl.npos, reinterpret_cast<cx<float>*>(f0node0), pa, Pl.d_status);
  } else {
    cx<double>* a = reinterpret_cast<cx<double>*>(Ai);
    hipLaunchKernelGGL((k_prep<double>), dim3(1), dim3(kThreads), 0, st, reinterpret_cast<const cx<double>*>(A),
                       reinterpret_cast<const cx<double>*>(b), reinterpret_cast<const cx<double>*>(c), a, a + n2,
                       a + n2 + Pl.npos, reinterpret_cast<cx<double>*>(f0node0), pa, Pl.d_status);
  }
  return hipGetLastError();
}

template <typename R>
static hipError_t run_forward_t(const Plan& Pl, bool odd, const void* A, const void* b, const void* c, void* rho,
                                char* ws, char* saved, hipStream_t st) {
  const bool store_all = saved != nullptr;
  // prep lives in the workspace; intermediates in `saved` (store-all) or the workspace (ring)
  FwdLayout Lw = fwd_layout(Pl, odd, false, 0);
  FwdLayout Ls = fwd_layout(Pl, true, true, 0);
  char* fb = store_all ? saved : ws;
  const FwdLayout& LF = store_all ? Ls : Lw;
  cx<R>* Ai = reinterpret_cast<cx<R>*>(ws + Lw.prep);
  cx<R>* bi = Ai + (size_t)Pl.npos * Pl.npos;
  cx<R>* ci = bi + Pl.npos;
  cx<R>* f0 = reinterpret_cast<cx<R>*>(fb + LF.f0);
  DevPlan P = make_devplan(Pl, odd);
  (void)ci;
  hipError_t e;
  {
    KTimer kt(Pl, KK_PREP, st);
    e = launch_prep(Pl, A, b, c, Ai, f0, st);
  }
  if (e != hipSuccess) return e;
  if (Pl.B > 1) {
    KTimer kt(Pl, KK_UFILL, st);
    const size_t shm = (size_t)Pl.B * sizeof(cx<R>);
    if (shm > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ufill<R>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL((k_ufill<R>), dim3(1), dim3(64), shm, st, P, Ai, bi, f0, Pl.d_elist, Pl.d_woff,
                       Pl.wmax);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (int S = 0; S <= Pl.smax && Pl.MD > 0; ++S) {
    LevelPtrs<R> L;
    std::memset(&L, 0, sizeof(L));
    for (int f = 1; f < Pl.nfam; ++f) {
      if (LF.fam[f] == 0) continue;
      const int g = Pl.fam_group[f];
      L.rd[f] = fam_level_ptr<R>(Pl, fb, LF.fam[f], g, S - 1, !store_all);
      L.wr[f] = fam_level_ptr<R>(Pl, fb, LF.fam[f], g, S, !store_all);
    }
    L.f0cur = fam_level_ptr<R>(Pl, fb, LF.f0, 0, S, false);
    L.f0nxt = S < Pl.smax ? fam_level_ptr<R>(Pl, fb, LF.f0, 0, S + 1, false) : nullptr;
    {
      KTimer kt(Pl, KK_FWD_LEVEL, st);
      e = launch_fwd_level_t<R>(Pl, P, odd, S, L, Ai, bi, st);
    }
    if (e != hipSuccess) return e;
  }
  if (!rho) return hipSuccess;   // recompute for the reverse sweep: no output needed
  const int64_t total = Pl.out_elems;
  const int64_t grid = std::min<int64_t>((total + kThreads - 1) / kThreads, 65536);
  const size_t shm = 16 * ((((size_t)(Pl.MD + 1) * (Pl.smax + 3)) * 4 + 15) / 16) + (size_t)(Pl.smax + 2) * 8;
  KTimer kt(Pl, KK_OUT_PERM, st);
  hipLaunchKernelGGL((k_out_perm<R>), dim3(grid), dim3(kThreads), shm, st, P, f0, reinterpret_cast<cx<R>*>(rho),
                     (int64_t)Pl.nodes_total, total, Pl.d_status);
  return hipGetLastError();
}

hipError_t run_forward(const Plan& Pl, bool odd, const void* A, const void* b, const void* c, void* rho, void* ws,
                       void* saved, hipStream_t st) {
  if (Pl.dt == FD_C64)
    return run_forward_t<float>(Pl, odd, A, b, c, rho, (char*)ws, (char*)saved, st);
  return run_forward_t<double>(Pl, odd, A, b, c, rho, (char*)ws, (char*)saved, st);
}

}  // namespace fd
