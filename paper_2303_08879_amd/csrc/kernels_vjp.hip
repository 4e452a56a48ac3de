// Reverse sweep (vector-Jacobian product) of the selective recurrence.
//
// Forward, every computed amplitude t has one canonical parent pivot p and
// direction i:  G_t = (b_i G_p + sum_l sqrt(p_l) A_il G_{p-1_l}) / sqrt(p_i+1)
// (Eq. recrel).  With h_t = gbar_t / sqrt(p_i + 1), the adjoint (Sec. 2.5,
// Eqs. dL_dB / dL_dA, in reverse instead of forward mode) is
//   gbar_{p-1_l} += sqrt(p_l) conj(A_il) h_t,   gbar_p += conj(b_i) h_t,
//   Abar_il      += conj(sqrt(p_l) G_{p-1_l}) h_t,   bbar_i += conj(G_p) h_t.
// The sweep visits the levels of the forward in reverse.  Each off-diagonal
// amplitude is read by exactly one pivot (Sec. 3.1.4 / App. B.2), so the
// cotangent slot of every read is *written* (not accumulated) by the thread
// of its only reader: no atomics, and two-level rings suffice for the
// cotangents.  Diagonal amplitudes F0(m) are read only by pivots that sit at
// the same lattice point m, so their cotangents are summed locally.
// Abar / bbar are sums over every target: each workgroup stages its
// per-pivot vectors (h, G-reads) in LDS and a fixed set of threads forms the
// outer products in a fixed order, then adds them to its own partial slot;
// one final kernel sums the slots in order.  The result is bitwise
// reproducible for a given plan.
#include <algorithm>
#include <cstring>

#include "vjp_common.h"

namespace fd {



template <typename R>
__global__ void k_zero_cx(cx<R>* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    st(p + i, czero<R>());
}

__global__ void k_zero_d2(double2* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_double2(0.0, 0.0);
}

// rho-shaped cotangent (C order [kappa][n_D]) -> node order (level-major)
template <typename R>
__global__ __launch_bounds__(kThreads) void k_perm_in(DevPlan P, const cx<R>* __restrict__ drho, cx<R>* __restrict__ g0,
                                                      int64_t N, int64_t total) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int* spn = reinterpret_cast<int*>(smem_raw);
  int64_t* slv = reinterpret_cast<int64_t*>(smem_raw + 16 * ((((P.MD + 1) * P.pnw) * 4 + 15) / 16));
  const int npn = (P.MD + 1) * P.pnw;
  for (int i = threadIdx.x; i < npn; i += blockDim.x) spn[i] = P.pn[i];
  for (int i = threadIdx.x; i <= P.smax; i += blockDim.x) slv[i] = P.MD > 0 ? P.lvl[i] : 0;
  __syncthreads();
  const int MD = P.MD, B = P.B, pnw = P.pnw;
  if (B > 1) {
    // tiles of kOutTN consecutive C-order lattice points n by kOutTK block
    // entries kappa through LDS, the inverse of the output permutation: each
    // kappa's run of n is read as one, each node's run of kappa written as one
    cx<R>* tl = reinterpret_cast<cx<R>*>(reinterpret_cast<unsigned char*>(slv) + 16 * (((P.smax + 2) * 8 + 15) / 16));
    constexpr int LD = kOutTK + 1;
    const int64_t ntn = (N + kOutTN - 1) / kOutTN, tiles = ntn * ((B + kOutTK - 1) / kOutTK);
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
      const int64_t n0 = (tile % ntn) * kOutTN;
      const int kap0 = (int)(tile / ntn) * kOutTK;
      {
        const int nl = threadIdx.x % kOutTN;
        for (int k = threadIdx.x / kOutTN; k < kOutTK; k += kThreads / kOutTN)
          if (n0 + nl < N && kap0 + k < B) tl[nl * LD + k] = ld(drho + (size_t)(kap0 + k) * N + n0 + nl);
      }
      __syncthreads();
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
          st(g0 + (size_t)(slv[S] + rank) * B + kap0 + kl, tl[nl * LD + kl]);
        }
      }
      __syncthreads();
    }
    return;
  }
  // one entry per node (no undetected modes): C-order index -> node order
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x)
    st(g0 + node_of_cindex(P, spn, slv, (int)idx), ld(drho + idx));
}

template <typename R>
__device__ __forceinline__ void load_tables_v(const DevPlan& P, int* spn, R* sq, R* isq) {
  const int n = (P.MD + 1) * P.pnw;
  for (int i = threadIdx.x; i < n; i += blockDim.x) spn[i] = P.pn[i];
  for (int v = threadIdx.x; v < kMaxCut + 4; v += blockDim.x) {
    sq[v] = sqrt(R(v));
    isq[v] = v ? R(1) / sqrt(R(v)) : R(0);
  }
}

// ---------------------------------------------------------------------------
// Algorithm 1 reverse step: one thread per lattice point.
// For each pivot the lane gathers the cotangents h of its targets, forms the
// adjoint of the reads (u = A^H h, with A and b read through uniform loads,
// so they live in scalar registers instead of LDS or vector registers) and
// writes the read cotangents.  The Abar / bbar records (h and the read
// values x, which only the reduction needs) are staged NB lanes at a time in
// the wave's LDS area and reduced on the matrix cores: a smaller batch keeps
// the staging area, and so the LDS per wave, small enough for several waves
// per SIMD; the read values of a lane are loaded when its batch is staged.
// ---------------------------------------------------------------------------
template <int MD, bool ODD, typename R, int NB>
__global__ __launch_bounds__(kThreads) void k_vjp_point(DevPlan P, VjpPtrs<R> V, const cx<R>* __restrict__ Ai,
                                                        const cx<R>* __restrict__ bi, int S, int nwork,
                                                        double2* __restrict__ partial) {
  constexpr int NP = 2 * MD;
  constexpr int NR = NP + 1;
  constexpr int NPAIR = NP * NR;
  constexpr int RS = NB + 1;   // padded row stride of the staging area
  static_assert(NB % 4 == 0 && 64 % NB == 0, "batches of whole MFMA steps that tile the wavefront");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<R>* rec = reinterpret_cast<cx<R>*>(smem_raw);                 // waves x RS x (NP + NR)
  R* sq = reinterpret_cast<R*>(rec + (size_t)(kThreads / 64) * RS * (NP + NR));
  R* isq = sq + (kMaxCut + 4);
  int* spn = reinterpret_cast<int*>(isq + (kMaxCut + 4));
  load_tables_v(P, spn, sq, isq);
  __syncthreads();
  cx<R>* recw = rec + (size_t)(threadIdx.x >> 6) * RS * (NP + NR);
  const int lane = threadIdx.x & 63;
  // columns of X that can be non-zero: the pivot value (bbar) only when odd
  // levels are swept
  constexpr int NCOL = ODD ? NR : NP;
  MfmaAcc<(NCOL + 15) / 16> acc;
  mfma_acc_zero(acc);
  const int pnw = P.pnw;

  for (int base = blockIdx.x * kThreads; base < nwork; base += gridDim.x * kThreads) {
    const int r = base + threadIdx.x;
    const bool live = r < nwork;
    int m[MD], s[MD + 1], rdn[MD], rup[MD];
#pragma unroll
    for (int d = 0; d < MD; ++d) m[d] = 0;
    int K0 = MD;
    cx<R> g0acc = czero<R>(), G0 = czero<R>();
    // the point's own F0 entry: always valid for a live lane, the address that
    // loads of absent neighbours or unset cotangent slots read instead (their
    // value is then discarded), so a pivot's loads are issued unconditionally
    // and share one wait
    const cx<R>* own = at32(V.fcur[0], (uint32_t)(live ? r : 0));
    if (live) {
      unrank<MD>(spn, pnw, P.CD, S, r, m, s);
      neighbour_ranks<MD>(spn, pnw, s, rdn, rup);
#pragma unroll
      for (int d = MD - 1; d >= 0; --d)
        if (m[d] > 0) K0 = d;
      g0acc = ld(at32(V.d0cur, (uint32_t)r));
      G0 = ld(own);
    }
    cx<R> ykg[MD];
#pragma unroll
    for (int K = 0; K < MD; ++K) ykg[K] = czero<R>();

#pragma unroll
    for (int K = 0; K < MD; ++K) {
      const bool valid = live && K <= K0 && m[K] <= P.CD[K] - 2;
      if (__ballot(valid) == 0ull) continue;   // uniform over the wave (each wave stages its own records)
      // the record's read values, loaded by every lane with the cotangents
      // (one memory round trip for both, and for both record batches)
      cx<R> xr[NCOL];
#pragma unroll
      for (int l = 0; l < NCOL; ++l) xr[l] = czero<R>();
      cx<R> h[NP];
#pragma unroll
      for (int i = 0; i < NP; ++i) h[i] = czero<R>();
      if (valid) {
        xr[2 * K] = cscale(G0, sq[m[K] + 1]);
        {
          const bool hk = m[K] > 0;
          const cx<R> v = ld(hk ? at32(V.fprev[fam_f2(MD, K)], (uint32_t)rdn[K]) : own);
          xr[2 * K + 1] = cscale(hk ? v : czero<R>(), sq[m[K]]);
        }
#pragma unroll
        for (int j = K + 1; j < MD; ++j) {
          const bool hj = m[j] > 0;
          const cx<R> v0 = ld(hj ? at32(V.fprev[fam_1001(MD, K, j)], (uint32_t)rdn[j]) : own);
          const cx<R> v1 = ld(hj ? at32(V.fprev[fam_1010(MD, K, j)], (uint32_t)rdn[j]) : own);
          xr[2 * j] = cscale(hj ? v0 : czero<R>(), sq[m[j]]);
          xr[2 * j + 1] = cscale(hj ? v1 : czero<R>(), sq[m[j]]);
        }
        if (ODD) xr[NP] = ld(at32(V.fcur[fam_f1k(K)], (uint32_t)r));
        // (no level above the last one under a total photon cutoff)
        if (V.gf0nxt) h[2 * K + 1] = cscale(ld(at32(V.gf0nxt, (uint32_t)rup[K])), isq[m[K] + 1]);
        {
          const bool t2 = m[K] <= P.CD[K] - 3;
          const cx<R> v = ld(t2 ? at32(V.gcur[fam_f2(MD, K)], (uint32_t)r) : own);
          h[2 * K] = cscale(t2 ? v : czero<R>(), isq[m[K] + 2]);
        }
#pragma unroll
        for (int j = K + 1; j < MD; ++j) {
          const bool tj = m[j] <= P.CD[j] - 2;
          const cx<R> v0 = ld(tj ? at32(V.gcur[fam_1010(MD, K, j)], (uint32_t)r) : own);
          const cx<R> v1 = ld(tj ? at32(V.gcur[fam_1001(MD, K, j)], (uint32_t)r) : own);
          h[2 * j] = cscale(tj ? v0 : czero<R>(), isq[m[j] + 1]);
          h[2 * j + 1] = cscale(tj ? v1 : czero<R>(), isq[m[j] + 1]);
        }
        // adjoint of the reads
#pragma unroll
        for (int l = 2 * K; l < NP; ++l) {
          cx<R> u = czero<R>();
#pragma unroll
          for (int i = 2 * K; i < NP; ++i) cfma_conj(u, ld(Ai + i * NP + l), h[i]);
          const int j = l >> 1;
          if (l == 2 * K) {
            g0acc = cadd(g0acc, cscale(u, sq[m[K] + 1]));
          } else if (l == 2 * K + 1) {
            if (m[K] > 0) st(at32(V.gprev[fam_f2(MD, K)], (uint32_t)rdn[K]), cscale(u, sq[m[K]]));
          } else if (m[j] > 0) {
            st(at32(V.gprev[(l & 1) ? fam_1010(MD, K, j) : fam_1001(MD, K, j)], (uint32_t)rdn[j]), cscale(u, sq[m[j]]));
          }
        }
        if (ODD) {
          cx<R> gp = czero<R>();
#pragma unroll
          for (int i = 2 * K; i < NP; ++i) cfma_conj(gp, ld(bi + i), h[i]);
          const bool has_diag_reader = (K > 0) || (m[0] + 1 <= P.CD[0] - 2);
          ykg[K] = has_diag_reader ? cadd(ld(at32(V.gcur[fam_f1k(K)], (uint32_t)r)), gp) : gp;
        }
      }
      // Abar records of this pivot, NB lanes at a time
#pragma unroll 1
      for (int q = 0; q < 64 / NB; ++q) {
        const bool grp = (lane / NB) == q;
        if (__ballot(valid && grp) == 0ull) continue;   // uniform over the wave
        if (grp) {
          const int col = lane - q * NB;
#pragma unroll
          for (int l = 0; l < NCOL; ++l) recw[(NP + l) * RS + col] = xr[l];
#pragma unroll
          for (int i = 0; i < NP; ++i) recw[i * RS + col] = h[i];
        }
        wave_sync();
        wave_accum_mfma<R, NP, NCOL, NB>(recw, acc);
        wave_sync();
      }
    }

    if (ODD) {
      const bool valid = live && m[0] <= P.CD[0] - 2;
      if (__ballot(valid) != 0ull) {
        cx<R> xr[NCOL];
#pragma unroll
        for (int l = 0; l < NCOL; ++l) xr[l] = czero<R>();
        if (valid) {
#pragma unroll
          for (int j = 0; j < MD; ++j) {
            const bool hj = m[j] > 0;
            const cx<R> v0 = ld(hj ? at32(V.fprev[fam_f1b(MD, j)], (uint32_t)rdn[j]) : own);
            const cx<R> v1 = ld(hj ? at32(V.fprev[fam_f1k(j)], (uint32_t)rdn[j]) : own);
            xr[2 * j] = cscale(hj ? v0 : czero<R>(), sq[m[j]]);
            xr[2 * j + 1] = cscale(hj ? v1 : czero<R>(), sq[m[j]]);
          }
          xr[NP] = G0;
        }
        cx<R> h[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) h[i] = czero<R>();
        if (valid) {
#pragma unroll
          for (int j = 0; j < MD; ++j) {
            const bool okk = j == 0 || m[j] <= P.CD[j] - 2;
            const bool kpiv = (j <= K0) && (m[j] <= P.CD[j] - 2);
            const bool okb = (j == 0) ? (m[0] <= P.CD[0] - 3) : (m[j] <= P.CD[j] - 2);
            const cx<R> vk = ld(okk && !kpiv ? at32(V.gcur[fam_f1k(j)], (uint32_t)r) : own);
            const cx<R> vb = ld(okb ? at32(V.gcur[fam_f1b(MD, j)], (uint32_t)r) : own);
            h[2 * j] = okk ? cscale(kpiv ? ykg[j] : vk, isq[m[j] + 1]) : czero<R>();
            h[2 * j + 1] = cscale(okb ? vb : czero<R>(), isq[m[j] + 1]);
          }
#pragma unroll
          for (int l = 0; l < NP; ++l) {
            const int j = l >> 1;
            if (m[j] == 0) continue;
            cx<R> u = czero<R>();
#pragma unroll
            for (int i = 0; i < NP; ++i) cfma_conj(u, ld(Ai + i * NP + l), h[i]);
            st(at32(V.gprev[(l & 1) ? fam_f1k(j) : fam_f1b(MD, j)], (uint32_t)rdn[j]), cscale(u, sq[m[j]]));
          }
          cx<R> gp = czero<R>();
#pragma unroll
          for (int i = 0; i < NP; ++i) cfma_conj(gp, ld(bi + i), h[i]);
          g0acc = cadd(g0acc, gp);
        }
#pragma unroll 1
        for (int q = 0; q < 64 / NB; ++q) {
          const bool grp = (lane / NB) == q;
          if (__ballot(valid && grp) == 0ull) continue;
          if (grp) {
            const int col = lane - q * NB;
#pragma unroll
            for (int l = 0; l < NCOL; ++l) recw[(NP + l) * RS + col] = xr[l];
#pragma unroll
            for (int i = 0; i < NP; ++i) recw[i * RS + col] = h[i];
          }
          wave_sync();
          wave_accum_mfma<R, NP, NCOL, NB>(recw, acc);
          wave_sync();
        }
      }
    }
    if (live) st(at32(V.gcur[0], (uint32_t)r), g0acc);
  }
  // fold the per-wave pair tables (fixed order) into this block's slot
  cx<double>* red = reinterpret_cast<cx<double>*>(smem_raw);
  __syncthreads();
  mfma_acc_store<NP, NR, NCOL>(acc, red + (size_t)(threadIdx.x >> 6) * NPAIR);
  __syncthreads();
  double2* slot = partial + (size_t)blockIdx.x * NPAIR;
  for (int p = threadIdx.x; p < NPAIR; p += blockDim.x) {
    if (p - (p / NR) * NR >= NCOL) continue;   // the bbar column without odd levels: zero
    double sx = 0.0, sy = 0.0;
    for (int wv = 0; wv < kThreads / 64; ++wv) {
      sx += red[(size_t)wv * NPAIR + p].x;
      sy += red[(size_t)wv * NPAIR + p].y;
    }
    const double2 v = slot[p];
    slot[p] = make_double2(v.x + sx, v.y + sy);
  }
}

// ---------------------------------------------------------------------------
// Reverse of step 1 of Algorithm 2 (undetected block at zero detections), by
// weight from the top, one wavefront with the block's forward values and
// cotangents in LDS: an entry's cotangent gathers from the targets that used
// it as pivot (x + 1_q with first non-zero coordinate q) or as a read
// (x + 1_q2 + 1_q with parent x + 1_q2, first non-zero coordinate q).
// As in the forward fill, every operand of the weight steps is staged in LDS
// first (incoming cotangents included), so the steps never wait on global
// memory.  LDS: ufill_lds_bytes(plan, true).
// ---------------------------------------------------------------------------
template <typename R, int NQ, bool ST = false>
__global__ __launch_bounds__(64) void k_ufill_vjp(DevPlan P, const cx<R>* __restrict__ Ai,
                                                  const cx<R>* __restrict__ bi, const cx<R>* __restrict__ G,
                                                  const cx<R>* __restrict__ gin, const int* __restrict__ elist,
                                                  const int* __restrict__ woff, int wmax, double2* slot,
                                                  cx<R>* cbar, cx<R>* gbuf) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int nq = NQ;   // 2 per undetected mode
  const int npos = P.npos, B = P.B;
  const int NR = npos + 1;
  const int lane = threadIdx.x;
  // forward values and cotangents of the block: in LDS, or (ST) read from
  // HBM where the forward left them and accumulated in `gbuf` (B entries of
  // the workspace)
  cx<R>* Gl = reinterpret_cast<cx<R>*>(smem_raw);
  cx<R>* gf = ST ? gbuf : Gl + B;
  cx<R>* sA = ST ? Gl : gf + B;   // A between undetected positions, row stride NQ
  cx<R>* sb = sA + NQ * NQ;
  R* sq = reinterpret_cast<R*>(sb + NQ);
  R* isq = sq + (kMaxCut + 4);
  const int* el = elist;
  const int* wo = woff;
  auto GL = [&](int i) -> cx<R> {
    if constexpr (ST)
      return ld(G + i);
    else
      return Gl[i];
  };
  if constexpr (ST) {
    for (int e = lane; e < B; e += 64) st(gf + e, ld(gin + e));
  } else {
    int* lel = reinterpret_cast<int*>(isq + (kMaxCut + 4));
    int* lwo = lel + B;
    for (int e = lane; e < B; e += 64) {
      Gl[e] = ld(G + e);
      gf[e] = ld(gin + e);
      lel[e] = elist[e];
    }
    for (int t = lane; t < wmax + 2; t += 64) lwo[t] = woff[t];
    el = lel;
    wo = lwo;
  }
  for (int i = lane; i < nq * nq; i += 64) sA[(i / nq) * NQ + i % nq] = ld(Ai + (i / nq) * npos + i % nq);
  if (lane < nq) sb[lane] = ld(bi + lane);
  for (int v = lane; v < kMaxCut + 4; v += 64) {
    sq[v] = sqrt(R(v));
    isq[v] = v ? R(1) / sqrt(R(v)) : R(0);
  }
  unit_sync<ST>();
  cx<double> ab[NQ][NQ + 1];
#pragma unroll
  for (int a = 0; a < NQ; ++a)
#pragma unroll
    for (int c = 0; c <= NQ; ++c) ab[a][c] = cmake<double>(0.0, 0.0);
  for (int w = wmax; w >= 0; --w) {
    const int t1 = wo[w + 1];
    for (int t = wo[w] + lane; t < t1; t += 64) {
      const int e = el[t];
      int x[NQ];
      int rem = e;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        x[q] = q < nq ? ucoord(P, rem, q) : 0;
        rem -= x[q] * (q < nq ? P.ustride[q] : 0);
      }
      // first non-zero coordinate, its stride and value, selected with
      // constant indices (a lane-dependent index into the plan's arrays
      // would fetch them from argument memory on every step)
      int first0 = nq, usf = 0, xf = 0;
#pragma unroll
      for (int q = NQ - 1; q >= 0; --q)
        if (q < nq && x[q] > 0) {
          first0 = q;
          usf = P.ustride[q];
          xf = x[q];
        }
      cx<R> acc = gf[e];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (q >= nq || q > first0) continue;
        if (x[q] + 1 < P.udims[q]) {
          const cx<R> ht = cscale(gf[e + P.ustride[q]], isq[x[q] + 1]);
          cfma_conj(acc, sb[q], ht);
        }
#pragma unroll
        for (int q2 = 0; q2 < NQ; ++q2) {
          if (q2 < q || q2 >= nq) continue;
          const int p2 = x[q2] + 1;                  // parent coordinate along q2
          const int pq = x[q] + (q2 == q ? 1 : 0);   // parent coordinate along q
          if (p2 >= P.udims[q2] || pq + 1 >= P.udims[q]) continue;
          const cx<R> ht = cscale(gf[e + P.ustride[q2] + P.ustride[q]], isq[pq + 1]);
          cx<R> u = czero<R>();
          cfma_conj(u, sA[q * NQ + q2], ht);
          acc = cadd(acc, cscale(u, sq[p2]));
        }
      }
      gf[e] = acc;
      if (e > 0) {
        // this entry as a target: parent x - 1_first0, direction first0
        const int qf = first0;
        const int pe = e - usf;
        const cx<R> h = cscale(acc, isq[xf]);
        const cx<R> gp = GL(pe);
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
          if (a != qf) continue;
          ab[a][NQ].x += (double)gp.x * h.x + (double)gp.y * h.y;
          ab[a][NQ].y += (double)gp.x * h.y - (double)gp.y * h.x;
#pragma unroll
          for (int q2 = 0; q2 < NQ; ++q2) {
            if (q2 >= nq) continue;
            const int pq2 = x[q2] - (q2 == qf ? 1 : 0);
            if (pq2 <= 0) continue;
            const cx<R> g2 = cscale(GL(pe - P.ustride[q2]), sq[pq2]);
            ab[a][q2].x += (double)g2.x * h.x + (double)g2.y * h.y;
            ab[a][q2].y += (double)g2.x * h.y - (double)g2.y * h.x;
          }
        }
      }
    }
    unit_sync<ST>();
  }
  // butterfly sums over the wavefront (fixed order), lane 0 adds to the slot
#pragma unroll
  for (int a = 0; a < NQ; ++a) {
#pragma unroll
    for (int c = 0; c <= NQ; ++c) {
      if (a >= nq || (c >= nq && c != NQ)) continue;   // uniform
      double vx = ab[a][c].x, vy = ab[a][c].y;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        vx += __shfl_xor(vx, off, 64);
        vy += __shfl_xor(vy, off, 64);
      }
      if (lane == 0) {
        const int p = a * NR + (c == NQ ? npos : c);
        double2 v = slot[p];
        slot[p] = make_double2(v.x + vx, v.y + vy);
      }
    }
  }
  if (lane == 0) st(cbar, gf[0]);
}

// Final: sum the partial slots in order, symmetrise Abar, scatter to the
// caller's block order (zero for dropped modes), write dc.
struct FinalArgs {
  int blk2pos[2 * kMaxModes];
  int M2, npos;
};

template <typename R>
__global__ __launch_bounds__(kThreads) void k_vjp_final(const double2* __restrict__ partial, FinalArgs a,
                                                        const cx<R>* __restrict__ cbar, cx<R>* dA, cx<R>* db,
                                                        cx<R>* dc) {
  __shared__ double2 red[kThreads];
  const int NR = a.npos + 1, P = a.npos * NR;
  const int idx = blockIdx.x;
  int c1 = -1, c2 = -1;   // pair columns summed (c2: transpose for the symmetric part)
  if (idx < a.M2 * a.M2) {
    const int p = a.blk2pos[idx / a.M2], q = a.blk2pos[idx % a.M2];
    if (p >= 0 && q >= 0) {
      c1 = p * NR + q;
      c2 = q * NR + p;
    }
  } else if (idx < a.M2 * a.M2 + a.M2) {
    const int p = a.blk2pos[idx - a.M2 * a.M2];
    if (p >= 0) c1 = p * NR + a.npos;
  }
  double sx = 0.0, sy = 0.0;
  // slots threadIdx.x, + kThreads, ... in order; a fixed trip count lets the
  // loads of all of them go out before the first add
  static_assert(kPartialSlots % kThreads == 0, "slot count");
  constexpr int KS = kPartialSlots / kThreads;
  if (c1 >= 0) {
    double2 v[KS], w[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const size_t s = threadIdx.x + (size_t)k * kThreads;
      v[k] = partial[s * P + c1];
      w[k] = c2 >= 0 ? partial[s * P + c2] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      sx += v[k].x;
      sy += v[k].y;
      if (c2 >= 0) {
        sx += w[k].x;
        sy += w[k].y;
      }
    }
  }
  red[threadIdx.x] = make_double2(sx, sy);
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[threadIdx.x].x += red[threadIdx.x + w].x;
      red[threadIdx.x].y += red[threadIdx.x + w].y;
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double2 t = red[0];
  if (idx < a.M2 * a.M2)
    st(dA + idx, cmake<R>((R)(0.5 * t.x), (R)(0.5 * t.y)));
  else if (idx < a.M2 * a.M2 + a.M2)
    st(db + (idx - a.M2 * a.M2), cmake<R>((R)t.x, (R)t.y));
  else
    st(dc, ld(cbar));
}

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------
template <typename R>
static const cx<R>* fptr(const Plan& Pl, const char* base, size_t off, int g, int S) {
  if (S < 0 || off == 0) return nullptr;
  return reinterpret_cast<const cx<R>*>(base + off +
                                         (size_t)Pl.lvl[(size_t)g * (Pl.smax + 2) + S] * Pl.B * sizeof(cx<R>));
}
template <typename R>
static cx<R>* gptr(const Plan& Pl, char* base, size_t off, int g, int S) {
  if (S < 0 || off == 0) return nullptr;
  return reinterpret_cast<cx<R>*>(base + off + (size_t)(S & 1) * Pl.maxN[g] * Pl.B * sizeof(cx<R>));
}

template <typename R>
static hipError_t run_vjp_t(const Plan& Pl, bool odd, const void* A, const void* b, const void* c,
                            const void* saved, const void* drho, void* dA, void* db, void* dc, char* ws,
                            hipStream_t st) {
  const VjpLayout V = vjp_layout(Pl, odd, 0);
  const FwdLayout Ls = fwd_layout(Pl, true, true, 0);
  const char* sv = reinterpret_cast<const char*>(saved);
  cx<R>* Ai = reinterpret_cast<cx<R>*>(ws + V.prep);
  cx<R>* bi = Ai + (size_t)Pl.npos * Pl.npos;
  cx<R>* cb = bi + Pl.npos;   // reused: holds cbar at the end
  double2* partial = reinterpret_cast<double2*>(ws + V.partial);
  hipError_t e;
  {
    KTimer kt(Pl, KK_PREP, st);
    e = launch_prep(Pl, A, b, c, Ai, nullptr, st);
  }
  if (e != hipSuccess) return e;
  const int PP = Pl.npos * (Pl.npos + 1);
  const int64_t npart = (int64_t)kPartialSlots * PP;
  {
    KTimer kt(Pl, KK_ZERO, st);
    hipLaunchKernelGGL(k_zero_d2, dim3((unsigned)std::min<int64_t>((npart + 255) / 256, 4096)), dim3(256), 0, st,
                       partial, npart);
  }
  DevPlan P = make_devplan(Pl, odd);
  cx<R>* g0 = reinterpret_cast<cx<R>*>(ws + V.g0);
  if (Pl.level_cap >= 0) {
    // a total photon cutoff: the cotangent already comes in level (node) order
    KTimer kt(Pl, KK_PERM_IN, st);
    if ((e = hipMemcpyAsync(g0, drho, (size_t)Pl.nodes_total * sizeof(cx<R>), hipMemcpyDeviceToDevice, st)) !=
        hipSuccess)
      return e;
  } else {
    const int64_t total = Pl.out_elems;
    const int64_t tiles = ((Pl.nodes_total + kOutTN - 1) / kOutTN) * ((Pl.B + kOutTK - 1) / kOutTK);
    const int64_t grid = std::min<int64_t>(Pl.B > 1 ? tiles : (total + kThreads - 1) / kThreads, 65536);
    const size_t shm = 16 * ((((size_t)(Pl.MD + 1) * (Pl.smax + 3)) * 4 + 15) / 16) +
                       16 * (((size_t)(Pl.smax + 2) * 8 + 15) / 16) +
                       (Pl.B > 1 ? (size_t)kOutTN * (kOutTK + 1) * sizeof(cx<R>) : 0);
    KTimer kt(Pl, KK_PERM_IN, st);
    hipLaunchKernelGGL((k_perm_in<R>), dim3(grid), dim3(kThreads), shm, st, P,
                       reinterpret_cast<const cx<R>*>(drho), g0, (int64_t)Pl.nodes_total, total);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int MD = Pl.MD;
  if (Pl.level_cap >= 0 && MD > 0) {
    // under a total photon cutoff the families of the last level feed no
    // target: their cotangents (read by that level's pivots) start at zero
    for (int f = 1; f < Pl.nfam; ++f) {
      if (V.gfam[f] == 0) continue;
      const int g = Pl.fam_group[f];
      const int64_t n = Pl.maxN[g] * Pl.B;
      hipLaunchKernelGGL((k_zero_cx<R>), dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, st,
                         gptr<R>(Pl, ws, V.gfam[f], g, Pl.smax), n);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  const size_t tab = 2 * (kMaxCut + 4) * sizeof(R) + (size_t)(MD + 1) * (Pl.smax + 3) * sizeof(int);
  // Checkpointed plans: the forward values of one segment of levels at a
  // time, recomputed from the segment's checkpoint into the segment buffer
  // (slot k holds level seg_lo - 1 + k); F0 of every level is in `saved`.
  const bool ck = Pl.ckpt > 0;
  const CkptLayout Lc = ck ? ckpt_layout(Pl) : CkptLayout();
  const SegLayout Sg = ck ? seg_layout(Pl) : SegLayout();
  const size_t f0off = ck ? Lc.f0 : Ls.f0;
  auto used = [&](int f) { return ckpt_keeps_family(Pl, f) && (odd || f >= 1 + 2 * MD); };
  // level L of family f in the segment buffer (levels seg_lo - 1 .. held)
  auto seg_slot = [&](int f, int lo, int L) {
    return reinterpret_cast<cx<R>*>(ws + Sg.fam[f] +
                                    (size_t)seg_node(Pl, Pl.fam_group[f], lo, L) * Pl.B * sizeof(cx<R>));
  };
  int seg_lo = Pl.smax + 1;
  for (int S = Pl.smax; S >= 0 && MD > 0; --S) {
    if (ck && S < seg_lo) {
      seg_lo = (S / Pl.ckpt) * Pl.ckpt;
      const int c = S / Pl.ckpt;
      if (c > 0) {
        const void* src[kMaxFam] = {};
        void* dst[kMaxFam] = {};
        int64_t n[kMaxFam] = {};
        for (int f = 1; f < Pl.nfam; ++f) {
          if (!used(f)) continue;
          src[f] = sv + Lc.ck[(size_t)(c - 1) * Pl.nfam + f];
          dst[f] = seg_slot(f, seg_lo, seg_lo - 1);
          n[f] = Pl.ncnt[(size_t)Pl.fam_group[f] * (Pl.smax + 1) + seg_lo - 1] * Pl.B;
        }
        if ((e = launch_copy_fams(Pl, src, dst, n, st)) != hipSuccess) return e;
      }
      const cx<R>* f0all = reinterpret_cast<const cx<R>*>(sv + f0off);
      for (int L = seg_lo; L <= S; ++L) {
        const void* rd[kMaxFam] = {};
        void* wr[kMaxFam] = {};
        for (int f = 1; f < Pl.nfam; ++f) {
          if (!used(f)) continue;
          rd[f] = L > 0 ? seg_slot(f, seg_lo, L - 1) : nullptr;
          wr[f] = seg_slot(f, seg_lo, L);
        }
        // F0 of level L + 1 is written again with the values it already holds
        cx<R>* f0nxt = L < Pl.smax ? const_cast<cx<R>*>(f0all) + (size_t)Pl.lvl[L + 1] * Pl.B : nullptr;
        KTimer kt(Pl, KK_FWD_LEVEL, st);
        if ((e = launch_fwd_level(Pl, odd, L, rd, wr, f0all + (size_t)Pl.lvl[L] * Pl.B, f0nxt, Ai, bi, st)) !=
            hipSuccess)
          return e;
      }
    }
    VjpPtrs<R> Vp;
    std::memset(&Vp, 0, sizeof(Vp));
    for (int f = 0; f < Pl.nfam; ++f) {
      const int g = Pl.fam_group[f];
      if (!ck || f == 0) {
        const size_t foff = f == 0 ? f0off : Ls.fam[f];
        Vp.fprev[f] = fptr<R>(Pl, sv, foff, g, S - 1);
        Vp.fcur[f] = fptr<R>(Pl, sv, foff, g, S);
      } else if (used(f)) {
        Vp.fprev[f] = S > 0 ? seg_slot(f, seg_lo, S - 1) : nullptr;
        Vp.fcur[f] = seg_slot(f, seg_lo, S);
      }
      Vp.gprev[f] = gptr<R>(Pl, ws, V.gfam[f], g, S - 1);
      Vp.gcur[f] = gptr<R>(Pl, ws, V.gfam[f], g, S);
    }
    Vp.gf0nxt = (Pl.level_cap >= 0 && S == Pl.smax) ? nullptr : gptr<R>(Pl, ws, V.gfam[0], 0, S + 1);
    // every level kernel reads these unconditionally
    if (!Vp.fcur[0] || !Vp.gcur[0]) return hipErrorInvalidValue;
    Vp.d0cur = reinterpret_cast<const cx<R>*>(reinterpret_cast<const char*>(g0) +
                                              (size_t)Pl.lvl[S] * Pl.B * sizeof(cx<R>));
    Vp.node = Pl.d_node ? Pl.d_node + (size_t)Pl.lvl[S] * kNodeStride : nullptr;
    Vp.priv = V.priv ? reinterpret_cast<cx<R>*>(ws + V.priv) : nullptr;
    Vp.priv_stride = (int64_t)vjp_private_entries(Pl);
    const int nwork = (int)Pl.ncnt[S];
    KTimer kt(Pl, KK_VJP_LEVEL, st);
    if (Pl.B == 1) {
      const int NP = 2 * MD;
      const size_t shm = std::max((size_t)(kThreads / 64) * (kPointBatch + 1) * (2 * NP + 1) * sizeof(cx<R>),
                                  (size_t)(kThreads / 64) * NP * (NP + 1) * sizeof(cx<double>)) + tab;
      const int grid = (int)std::min<int64_t>((nwork + kThreads - 1) / kThreads, kPartialSlots - 1);
#define FD_VJP_POINT(MDV)                                                                                        \
  case MDV:                                                                                                      \
    if (odd) {                                                                                                   \
      if (shm > 65536)                                                                                           \
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_vjp_point<MDV, true, R, kPointBatch>),       \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);                         \
      hipLaunchKernelGGL((k_vjp_point<MDV, true, R, kPointBatch>), dim3(grid), dim3(kThreads), shm, st, P, Vp, \
                         Ai, bi, S, nwork, partial);                                                             \
    } else {                                                                                                     \
      if (shm > 65536)                                                                                           \
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_vjp_point<MDV, false, R, kPointBatch>),      \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);                         \
      hipLaunchKernelGGL((k_vjp_point<MDV, false, R, kPointBatch>), dim3(grid), dim3(kThreads), shm, st, P,    \
                         Vp, Ai, bi, S, nwork, partial);                                                         \
    }                                                                                                            \
    break;
      switch (MD) {
        FD_VJP_POINT(1)
        FD_VJP_POINT(2)
        FD_VJP_POINT(3)
        FD_VJP_POINT(4)
        FD_VJP_POINT(5)
        FD_VJP_POINT(6)
        FD_VJP_POINT(7)
        FD_VJP_POINT(8)
        default:
          return hipErrorInvalidValue;
      }
#undef FD_VJP_POINT
    } else {
      if ((e = launch_vjp_block_level<R>(Pl, P, Vp, Ai, bi, S, nwork, partial, st)) != hipSuccess) return e;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // cotangent of the seed block: F0 ring slot of level 0 (MD > 0) or drho itself
  const cx<R>* gseed = MD > 0 ? gptr<R>(Pl, ws, V.gfam[0], 0, 0) : g0;
  const cx<R>* cbar_src = gseed;
  if (Pl.B > 1) {
    const cx<R>* G0blk = reinterpret_cast<const cx<R>*>(sv + f0off);
    KTimer kt(Pl, KK_UFILL_VJP, st);
    const size_t shm = ufill_launch_lds_bytes(Pl, true);
    if (shm > kMaxLds) return hipErrorInvalidConfiguration;
    // streamed: the block's cotangents accumulate in the workspace
    cx<R>* gbuf = Pl.st_ufill_vjp ? reinterpret_cast<cx<R>*>(ws + V.ublk) : nullptr;
    if (Pl.st_ufill_vjp && V.ublk == 0) return hipErrorInvalidValue;
    auto* kfn = Pl.st_ufill_vjp ? (Pl.nq == 2   ? &k_ufill_vjp<R, 2, true>
                                   : Pl.nq == 4 ? &k_ufill_vjp<R, 4, true>
                                                : &k_ufill_vjp<R, 6, true>)
                                : (Pl.nq == 2   ? &k_ufill_vjp<R, 2, false>
                                   : Pl.nq == 4 ? &k_ufill_vjp<R, 4, false>
                                                : &k_ufill_vjp<R, 6, false>);
    if (shm > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kfn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm);
    hipLaunchKernelGGL(kfn, dim3(1), dim3(64), shm, st, P, Ai, bi, G0blk, gseed, Pl.d_elist, Pl.d_woff, Pl.wmax,
                       partial + (size_t)(kPartialSlots - 1) * PP, cb, gbuf);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    cbar_src = cb;
  }
  FinalArgs fa;
  std::memset(&fa, 0, sizeof(fa));
  for (int u = 0; u < 2 * Pl.M; ++u) fa.blk2pos[u] = -1;
  for (int p = 0; p < Pl.npos; ++p) fa.blk2pos[Pl.pos2blk[p]] = p;
  fa.M2 = 2 * Pl.M;
  fa.npos = Pl.npos;
  const int nout = fa.M2 * fa.M2 + fa.M2 + 1;
  KTimer kt(Pl, KK_VJP_FINAL, st);
  hipLaunchKernelGGL((k_vjp_final<R>), dim3(nout), dim3(kThreads), 0, st, partial, fa, cbar_src,
                     reinterpret_cast<cx<R>*>(dA), reinterpret_cast<cx<R>*>(db), reinterpret_cast<cx<R>*>(dc));
  return hipGetLastError();
}

hipError_t run_vjp(const Plan& Pl, bool odd, const void* A, const void* b, const void* c, const void* saved,
                   const void* drho, void* dA, void* db, void* dc, void* ws, hipStream_t st) {
  if (Pl.dt == FD_C64) return run_vjp_t<float>(Pl, odd, A, b, c, saved, drho, dA, db, dc, (char*)ws, st);
  return run_vjp_t<double>(Pl, odd, A, b, c, saved, drho, dA, db, dc, (char*)ws, st);
}

}  // namespace fd
