// Per-unit device code of the forward sweep, shared by the per-circuit level
// kernels and the batched persistent kernel.
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
// units are pure gathers with no atomics.  All targets of one step are
// independent (Sec. 2.2, the two parallelisations).
//
// `LP` is any type with L.rd[f] / L.wr[f] (node-0 pointers of family f at the
// levels S-1 / S) and L.f0cur / L.f0nxt (F0 at levels S / S+1).
#pragma once

#include "fd_device.h"

namespace fd {

static_assert(kBT == 64, "kBT is one wavefront");

// ---------------------------------------------------------------------------
// prep: caller's triple (block order) -> interleaved internal positions,
// A symmetrised; input finiteness and the b = 0 promise checked on device.
// ---------------------------------------------------------------------------
struct PrepArgs {
  int pos2blk[kMaxPos];
  int npos, M2, check_b_zero;
};

template <typename R>
__device__ __forceinline__ void prep_body(const cx<R>* __restrict__ A, const cx<R>* __restrict__ b,
                                          const cx<R>* __restrict__ c, cx<R>* __restrict__ Ai,
                                          cx<R>* __restrict__ bi, cx<R>* __restrict__ ci,
                                          cx<R>* __restrict__ f0node0, const PrepArgs& a, int* status) {
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

// Debug write counter of an amplitude written at dst: counter k of the
// store-all buffer's element k (fd_plan_set_write_counters, a check of the
// exactly-once writes of Sec. 3.1.4); a no-op when the counters are off.
template <typename R>
__device__ __forceinline__ void count_write(const DevPlan& P, const cx<R>* dst) {
  if (P.wcnt == nullptr) return;
  const int64_t k = (int64_t)(reinterpret_cast<const char*>(dst) - P.wbase) / (int64_t)sizeof(cx<R>);
  if (k >= 0 && k < P.wcnt_n) atomicAdd(P.wcnt + k, 1u);
}

// ---------------------------------------------------------------------------
// Step 1 of Algorithm 2: the whole undetected block at zero detections.
// Entry kappa != 0 is pulled from its parent kappa - 1_q, q = first non-zero
// coordinate, by Eq. recrel restricted to the undetected positions.  One
// wavefront, the block in LDS, entries visited by weight (host-built list).
// The weights form a chain of dependent steps, so everything a step reads
// (entry list, A and b between undetected positions, square-root tables) is
// staged in LDS first and a step never waits on global memory.
// LDS: ufill_lds_bytes(plan, false) (E = cx<R>); the forward mode carries
// value and tangent (E = dual<R>) through the same steps.
// ---------------------------------------------------------------------------
template <typename R, int NQ, typename E, bool ST = false>
__device__ __forceinline__ void ufill_body(const DevPlan& P, const cx<R>* __restrict__ Ai,
                                           const cx<R>* __restrict__ bi, cx<R>* G, const int* __restrict__ elist,
                                           const int* __restrict__ woff, int wmax, E* g, int64_t dT = 0) {
  using T = ET<E>;
  static_assert(!ST || std::is_same<E, cx<R>>::value, "the streamed fill carries values only");
  constexpr int nq = NQ;   // 2 per undetected mode
  const int npos = P.npos, B = P.B;
  const int lane = threadIdx.x & 63;
  // the block: in LDS, or (ST) the node-0 block itself in HBM
  E* blk;
  E* sA;   // A between undetected positions, row stride NQ
  if constexpr (ST) {
    blk = reinterpret_cast<E*>(G);
    sA = g;
  } else {
    blk = g;
    sA = g + B;
  }
  E* sb = sA + NQ * NQ;
  R* sq = reinterpret_cast<R*>(sb + NQ);
  R* isq = sq + (kMaxCut + 4);
  const int* el = elist;
  const int* wo = woff;
  if constexpr (!ST) {
    int* lel = reinterpret_cast<int*>(isq + (kMaxCut + 4));
    int* lwo = lel + B;
    for (int t = lane; t < B; t += 64) lel[t] = elist[t];
    for (int t = lane; t < wmax + 2; t += 64) lwo[t] = woff[t];
    el = lel;
    wo = lwo;
  }
  for (int i = lane; i < nq * nq; i += 64) sA[(i / nq) * NQ + i % nq] = T::load(Ai + (i / nq) * npos + i % nq, dT);
  if (lane < nq) sb[lane] = T::load(bi + lane, dT);
  for (int v = lane; v < kMaxCut + 4; v += 64) {
    sq[v] = sqrt(R(v));
    isq[v] = v ? R(1) / sqrt(R(v)) : R(0);
  }
  if constexpr (!ST)
    if (lane == 0) blk[0] = T::load(G, dT);   // c, written by the prep kernel
  unit_sync<ST>();
  for (int w = 1; w <= wmax; ++w) {
    const int t1 = wo[w + 1];
    for (int t = wo[w] + lane; t < t1; t += 64) {
      const int e = el[t];
      int kap[NQ];
      int rem = e;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        kap[q] = q < nq ? ucoord(P, rem, q) : 0;
        rem -= kap[q] * (q < nq ? P.ustride[q] : 0);
      }
      // first non-zero coordinate, its stride and value (selected with
      // constant indices: a lane-dependent index into the plan's arrays
      // would fetch them from argument memory on every step)
      int qf = nq, usf = 0, kqf = 0;
#pragma unroll
      for (int q = NQ - 1; q >= 0; --q)
        if (q < nq && kap[q] > 0) {
          qf = q;
          usf = P.ustride[q];
          kqf = kap[q];
        }
      const int pe = e - usf;
      E acc = T::zero();
      cfma(acc, sb[qf], blk[pe]);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (q >= nq) continue;
        const int pq = kap[q] - (q == qf ? 1 : 0);
        if (pq > 0) cfma(acc, sA[qf * NQ + q], cscale(blk[pe - P.ustride[q]], sq[pq]));
      }
      blk[e] = cscale(acc, isq[kqf]);
      if constexpr (ST) count_write(P, G + e);
    }
    unit_sync<ST>();
  }
  // entry 0 is the seed c, already in G (written by the prep kernel)
  if constexpr (!ST)
    for (int e = lane; e < B; e += 64)
      if (e > 0) {
        T::store(G + e, blk[e], dT);
        count_write(P, G + e);
      }
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
template <int MD, bool ODD, typename R, typename LP>
__device__ __forceinline__ void fwd_point_unit(const DevPlan& P, const LP& L, const cx<R>* __restrict__ Ai,
                                               const cx<R>* __restrict__ bi, const int* spn, const R* sq,
                                               const R* isq, int S, int r) {
  constexpr int NP = 2 * MD;
  const int pnw = P.pnw;
  int m[MD], s[MD + 1], rdn[MD], rup[MD];
  unrank<MD>(spn, pnw, P.CD, S, r, m, s);
  neighbour_ranks<MD>(spn, pnw, s, rdn, rup);

  // the point's own F0 entry: always valid, the address that neighbour loads
  // of absent neighbours read instead (their value is then discarded), so
  // every load is issued unconditionally and a pivot's loads share one wait
  const cx<R>* own = at32(L.f0cur, (uint32_t)r);
  const cx<R> g0 = ld(own);
  cx<R> yk[MD];
#pragma unroll
  for (int K = 0; K < MD; ++K) yk[K] = czero<R>();

  if (ODD && m[0] <= P.CD[0] - 2) {
    // diagonal pivot d(m): reads d(m) - 1_l, writes d(m) + 1_i (type-1 offsets)
    cx<R> x[NP];
#pragma unroll
    for (int j = 0; j < MD; ++j) {
      const bool h = m[j] > 0;
      const cx<R> vb = ld(h ? at32(L.rd[fam_f1b(MD, j)], (uint32_t)rdn[j]) : own);   // d(m)-1_ket(j) = F1b(j)(m-1_j)
      const cx<R> vk = ld(h ? at32(L.rd[fam_f1k(j)], (uint32_t)rdn[j]) : own);      // d(m)-1_bra(j) = F1k(j)(m-1_j)
      x[2 * j] = cscale(h ? vb : czero<R>(), sq[m[j]]);
      x[2 * j + 1] = cscale(h ? vk : czero<R>(), sq[m[j]]);
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
          if (j == 0 || m[j] <= P.CD[j] - 2) {
            cx<R>* dst = at32(L.wr[fam_f1k(j)], (uint32_t)r);
            st(dst, acc);
            count_write(P, dst);
          }
        } else {
          const bool ok = (j == 0) ? (m[0] <= P.CD[0] - 3) : (m[j] <= P.CD[j] - 2);
          if (ok) {
            cx<R>* dst = at32(L.wr[fam_f1b(MD, j)], (uint32_t)r);
            st(dst, acc);
            count_write(P, dst);
          }
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
    {
      const bool h = m[K] > 0;
      const cx<R> v = ld(h ? at32(L.rd[fam_f2(MD, K)], (uint32_t)rdn[K]) : own);
      x[2 * K + 1] = cscale(h ? v : czero<R>(), sq[m[K]]);
    }
#pragma unroll
    for (int j = K + 1; j < MD; ++j) {
      const bool h = m[j] > 0;
      const cx<R> v0 = ld(h ? at32(L.rd[fam_1001(MD, K, j)], (uint32_t)rdn[j]) : own);
      const cx<R> v1 = ld(h ? at32(L.rd[fam_1010(MD, K, j)], (uint32_t)rdn[j]) : own);
      x[2 * j] = cscale(h ? v0 : czero<R>(), sq[m[j]]);
      x[2 * j + 1] = cscale(h ? v1 : czero<R>(), sq[m[j]]);
    }
    // writes p + 1_i
#pragma unroll
    for (int i = 2 * K; i < NP; ++i) {
      const int j = i >> 1;
      bool ok;
      R scale;
      cx<R>* dst;
      if (i == 2 * K + 1) {                 // d(m + 1_K): output amplitude
        ok = L.f0nxt != nullptr;            // none above the last level (a total photon cutoff)
        scale = isq[m[K] + 1];
        dst = at32(L.f0nxt, (uint32_t)rup[K]);
      } else if (i == 2 * K) {              // F2(K)(m)
        ok = (m[K] <= P.CD[K] - 3);
        scale = isq[m[K] + 2];
        dst = at32(L.wr[fam_f2(MD, K)], (uint32_t)r);
      } else {                              // F1010(K,j)(m) / F1001(K,j)(m)
        ok = (m[j] <= P.CD[j] - 2);
        scale = isq[m[j] + 1];
        dst = at32(L.wr[(i & 1) ? fam_1001(MD, K, j) : fam_1010(MD, K, j)], (uint32_t)r);
      }
      if (!ok) continue;
      cx<R> acc = czero<R>();
      if (ODD) cfma(acc, ld(bi + i), yk[K]);
#pragma unroll
      for (int l = 2 * K; l < NP; ++l) cfma(acc, ld(Ai + i * NP + l), x[l]);
      st(dst, cscale(acc, scale));
      count_write(P, dst);
    }
  }
}

// ---------------------------------------------------------------------------
// Algorithm 2 (undetected modes present).  A node's block of B entries is
// split into chunks of whole rows of the first undetected coordinate (rows of
// R0 = B / C0 entries); the WV wavefronts of one workgroup handle one
// (lattice point, chunk); the batched sweep gives each unit one wavefront.
// The pivot's undetected neighbours reach one row back, so a chunk computes
// the pivot rows it needs one row above its own (recomputed, not stored).
// LDS: F0(m) rows [k0-2, k1) and the bridge pivot blocks F1k(K)(m), rows
// [k0-1, k1), for every bridge K applied at m.  ST (blocks whose rows do not
// fit the LDS): F0(m) is read from HBM where it lies and lpk is the
// workgroup's slot in global memory; workgroup-scope fences order its
// writes before other lanes read them.
// ---------------------------------------------------------------------------
template <int MD, int NQ, typename R, typename LP, typename E, bool ST = false, int WV = 1>
__device__ __forceinline__ void fwd_block_unit(const DevPlan& P, const LP& L, const E* sA, const E* sb,
                                               const R* sq, const R* isq, int S, int r, int c, const ChunkGeo& G,
                                               E* lf0, E* lpk, int64_t dT = 0) {
  using T = ET<E>;
  constexpr int NPD = 2 * MD;
  constexpr int NPOS = NQ + NPD;
  // Fences between loop iterations for the shapes whose unfenced build needs
  // more than 168 VGPRs (two waves per SIMD): there they lift occupancy by one
  // or two waves.  Where the unfenced unit already runs three waves, the
  // overlap of iterations is worth more than a fourth wave.
  constexpr bool kFence = MD >= 4 || (MD >= 3 && NQ >= 4);
  const int B = P.B, R0 = G.R0;
  // WV wavefronts share the unit (the lanes of the whole workgroup)
  constexpr int NT = kBT * WV;
  constexpr bool kBar = ST || WV > 1;
  const int lane = WV == 1 ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
  const int pk1 = (G.RC + 1) * R0;   // entries of one pivot block in LDS
  {
    const int k0 = c * G.RC, k1 = min(G.C0, k0 + G.RC);
    int m[MD], rdn[MD], rup[MD];
    node_record<MD>(L.node, r, m, rdn, rup);
    int K0 = MD;
#pragma unroll
    for (int d = MD - 1; d >= 0; --d)
      if (m[d] > 0) K0 = d;
    if (m[0] > P.CD[0] - 2) return;   // no pivot at this point (uniform)
    // F0(m), rows [k0-2, k1): entry e of the node's block
    const int f0base = (k0 - 2) * R0;
    const cx<R>* f0g = at32(L.f0cur, (uint32_t)(r * B));
    auto F0 = [&](int e) -> E {
      if constexpr (ST)
        return T::load(at32(f0g, (uint32_t)e), dT);
      else
        return lf0[e - f0base];
    };
    if constexpr (!ST) {
      const int e0 = max(0, k0 - 2) * R0, e1 = k1 * R0;
      for (int e = e0 + lane; e < e1; e += NT) lf0[e - f0base] = T::load(at32(f0g, (uint32_t)e), dT);
    }
    unit_sync<kBar>();
    // diagonal pivot, rows [k0-1, k1): own rows store every type-1 target,
    // the halo row only keeps the bridge pivot blocks
    {
      const int e0 = max(0, k0 - 1) * R0, e1 = k1 * R0;
      for (int e = e0 + lane; e < e1; e += NT) {
        const bool own = e >= k0 * R0;
        int kap[NQ];
        int rem = e;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          kap[q] = ucoord(P, rem, q);
          rem -= kap[q] * P.ustride[q];
        }
        const E piv = F0(e);
        E un[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) un[q] = kap[q] > 0 ? cscale(F0(e - P.ustride[q]), sq[kap[q]]) : T::zero();
        E x[NPD];
#pragma unroll
        for (int j = 0; j < MD; ++j) {
          if (m[j] > 0) {
            x[2 * j] = cscale(T::load(at32(L.rd[fam_f1b(MD, j)], (uint32_t)(rdn[j] * B + e)), dT), sq[m[j]]);
            x[2 * j + 1] = cscale(T::load(at32(L.rd[fam_f1k(j)], (uint32_t)(rdn[j] * B + e)), dT), sq[m[j]]);
          } else {
            x[2 * j] = T::zero();
            x[2 * j + 1] = T::zero();
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
            E acc = T::zero();
            cfma(acc, sb[NQ + i], piv);
#pragma unroll
            for (int q = 0; q < NQ; ++q) cfma(acc, sA[row + q], un[q]);
#pragma unroll
            for (int l = 0; l < NPD; ++l) cfma(acc, sA[row + NQ + l], x[l]);
            acc = cscale(acc, isq[m[j] + 1]);
            if (ok && own) {
              cx<R>* dst = at32(L.wr[side ? fam_f1b(MD, j) : fam_f1k(j)], (uint32_t)(r * B + e));
              T::store(dst, acc, dT);
              count_write(P, dst);
            }
            if (bridge) lpk[(size_t)j * pk1 + (e - (k0 - 1) * R0)] = acc;
          }
        }
        if constexpr (kFence) compiler_fence();
      }
    }
    unit_sync<kBar>();
    // bridges d(m) + 1_ket(K), own rows
#pragma unroll
    for (int K = 0; K < MD; ++K) {
      if (K > K0 || m[K] > P.CD[K] - 2) continue;   // uniform
      const E* pv = lpk + (size_t)K * pk1;
      for (int e = k0 * R0 + lane; e < k1 * R0; e += NT) {
        int kap[NQ];
        int rem = e;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          kap[q] = ucoord(P, rem, q);
          rem -= kap[q] * P.ustride[q];
        }
        const int lp = e - (k0 - 1) * R0;
        const E piv = pv[lp];
        E un[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) un[q] = kap[q] > 0 ? cscale(pv[lp - P.ustride[q]], sq[kap[q]]) : T::zero();
        E x[NPD];
        x[2 * K] = cscale(F0(e), sq[m[K] + 1]);
        x[2 * K + 1] = (m[K] > 0) ? cscale(T::load(at32(L.rd[fam_f2(MD, K)], (uint32_t)(rdn[K] * B + e)), dT), sq[m[K]]) : T::zero();
#pragma unroll
        for (int j = K + 1; j < MD; ++j) {
          if (m[j] > 0) {
            x[2 * j] = cscale(T::load(at32(L.rd[fam_1001(MD, K, j)], (uint32_t)(rdn[j] * B + e)), dT), sq[m[j]]);
            x[2 * j + 1] = cscale(T::load(at32(L.rd[fam_1010(MD, K, j)], (uint32_t)(rdn[j] * B + e)), dT), sq[m[j]]);
          } else {
            x[2 * j] = T::zero();
            x[2 * j + 1] = T::zero();
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
            dst = at32(L.f0nxt, (uint32_t)(rup[K] * B + e));
          } else if (i == 2 * K) {
            ok = (m[K] <= P.CD[K] - 3);
            scale = isq[m[K] + 2];
            dst = at32(L.wr[fam_f2(MD, K)], (uint32_t)(r * B + e));
          } else {
            ok = (m[j] <= P.CD[j] - 2);
            scale = isq[m[j] + 1];
            dst = at32(L.wr[(i & 1) ? fam_1001(MD, K, j) : fam_1010(MD, K, j)], (uint32_t)(r * B + e));
          }
          if (!ok) continue;
          const int row = (NQ + i) * NPOS;
          E acc = T::zero();
          cfma(acc, sb[NQ + i], piv);
#pragma unroll
          for (int q = 0; q < NQ; ++q) cfma(acc, sA[row + q], un[q]);
#pragma unroll
          for (int l = 2 * K; l < NPD; ++l) cfma(acc, sA[row + NQ + l], x[l]);
          T::store(dst, cscale(acc, scale), dT);
          count_write(P, dst);
        }
        if constexpr (kFence) compiler_fence();
      }
      if constexpr (kFence) compiler_fence();
    }
    unit_sync<kBar>();
  }
}

// ---------------------------------------------------------------------------
// F0 -> rho for plans without undetected modes (one entry per node): the
// value of output element idx, C order over the detected modes (spn = PN
// table, slv = level node offsets of F0).
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ cx<R> out_perm_elem(const DevPlan& P, const int* spn, const int64_t* slv,
                                               const cx<R>* __restrict__ f0, int64_t N, int64_t idx) {
  (void)N;
  return ld(f0 + node_of_cindex(P, spn, slv, (int)idx));
}

// F0 -> rho for plans with undetected modes, one tile of kOutTN consecutive
// C-order lattice points n by kOutTK consecutive block entries kappa, through
// LDS: every node's kOutTK entries are read as one contiguous run and every
// kappa's kOutTN outputs written as one (the element-wise gather reads a
// 64-byte sector per 16-byte element).  256 threads; returns 1 if a
// non-finite value was stored.
template <typename R>
__device__ __forceinline__ int out_perm_tile(const DevPlan& P, const int* spn, const int64_t* slv,
                                             const cx<R>* __restrict__ f0, cx<R>* __restrict__ rho, int64_t N,
                                             int64_t tile, cx<R>* tl) {
  const int MD = P.MD, B = P.B, pnw = P.pnw;
  const int64_t ntn = (N + kOutTN - 1) / kOutTN;
  const int64_t tn = tile % ntn, tk = tile / ntn;
  const int64_t n0 = tn * kOutTN;
  const int kap0 = (int)tk * kOutTK;
  constexpr int LD = kOutTK + 1;   // padded row: the column reads of the write phase spread over banks
  const int kl = threadIdx.x % kOutTK;
  for (int nl = threadIdx.x / kOutTK; nl < kOutTN; nl += kThreads / kOutTK) {
    const int64_t n = n0 + nl;
    if (n < N && kap0 + kl < B) {
      int64_t rem = n;
      int v[kMaxD];
      int S = 0;
      for (int d = MD - 1; d >= 0; --d) {
        v[d] = (int)(rem % P.CD[d]);
        rem /= P.CD[d];
        S += v[d];
      }
      int rank = 0, sd = S;
      for (int d = 0; d < MD; ++d) {
        rank += pnv(spn, pnw, d + 1, sd) - pnv(spn, pnw, d + 1, sd - v[d]);
        sd -= v[d];
      }
      tl[nl * LD + kl] = ld(f0 + (size_t)(slv[S] + rank) * B + kap0 + kl);
    }
  }
  __syncthreads();
  int bad = 0;
  const int nl = threadIdx.x % kOutTN;
  for (int k = threadIdx.x / kOutTN; k < kOutTK; k += kThreads / kOutTN) {
    if (n0 + nl < N && kap0 + k < B) {
      const cx<R> v = tl[nl * LD + k];
      if (!isfinite(v.x) || !isfinite(v.y)) bad = 1;
      st(rho + (size_t)(kap0 + k) * N + n0 + nl, v);
    }
  }
  __syncthreads();
  return bad;
}

}  // namespace fd
