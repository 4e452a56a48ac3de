// State vectors of pure Gaussian states: psi[n] = <n|psi> for 0 <= n_j < C_j.
//
// The generating function of a pure state has one index per mode (D = M in
// Sec. 2.1), and its scaled Taylor coefficients obey the same recurrence as
// the density matrix's:
//   psi[n] = ( b_i psi[p] + sum_l sqrt(p_l) A_il psi[p - 1_l] ) / sqrt(n_i),
// p = n - 1_i, taken here with i the first mode where n_i > 0.  Targets of
// total photon number S read levels S - 1 and S - 2 only, so the sweep runs
// level by level over the lattice of n (the detected lattice of a plan whose
// modes are all detected: same rank / unrank tables, same level-major
// storage, same output permutation).  With b = 0 the odd levels vanish
// (Sec. 2.4): even levels read level S - 2 alone and odd levels are only
// cleared.
//
// One thread per target; its parent's rank is rdn[i] of the target, its
// parent's own neighbour ranks come from the parent's partial sums (those of
// the target less one up to mode i).
#include <algorithm>
#include <cstring>
#include <vector>

#include "fd_device.h"

namespace fd {

struct StateModes {
  int MD;               // kept modes (cutoff >= 2)
  int mode[kMaxD];      // kept mode k -> caller's mode index
};

// A (symmetrised, (A + A^T)/2, as for density matrices) and b of the kept
// modes into the workspace (MD x MD, then MD), psi at the vacuum = c;
// non-finite inputs set status bit 0, a non-zero b under the b = 0 promise
// status bit 1.
template <typename R>
__global__ __launch_bounds__(64) void k_state_prep(int M, StateModes sm, const cx<R>* __restrict__ A,
                                                   const cx<R>* __restrict__ b, const cx<R>* __restrict__ c,
                                                   cx<R>* __restrict__ Ak, cx<R>* __restrict__ psi0, int check_b_zero,
                                                   int* status) {
  const int MD = sm.MD;
  int bad = 0;
  for (int i = threadIdx.x; i < MD * MD; i += blockDim.x) {
    const cx<R> v = ld(A + (size_t)sm.mode[i / MD] * M + sm.mode[i % MD]);
    const cx<R> w = ld(A + (size_t)sm.mode[i % MD] * M + sm.mode[i / MD]);
    if (!isfinite(v.x) || !isfinite(v.y)) bad |= 1;
    st(Ak + i, cmake<R>(R(0.5) * (v.x + w.x), R(0.5) * (v.y + w.y)));
  }
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    const cx<R> v = ld(b + i);
    if (!isfinite(v.x) || !isfinite(v.y)) bad |= 1;
    if (check_b_zero && (v.x != R(0) || v.y != R(0))) bad |= 2;
  }
  for (int i = threadIdx.x; i < MD; i += blockDim.x) st(Ak + MD * MD + i, ld(b + sm.mode[i]));
  if (threadIdx.x == 0) {
    const cx<R> cv = ld(c);
    if (!isfinite(cv.x) || !isfinite(cv.y)) bad |= 1;
    st(psi0, cv);
  }
  if (bad) atomicOr(status, bad);
}

// Level S of the sweep (S >= 1; S < 0: none) and, when zlevel >= 0, the
// clearing of level zlevel (an odd level under b = 0).  f0 is psi in level
// order; lvl[S] is the first entry of level S.
template <int MD, bool BZ, typename R>
__global__ __launch_bounds__(kThreads) void k_state_level(DevPlan P, const cx<R>* __restrict__ Ak,
                                                          cx<R>* __restrict__ f0, int S, int zlevel) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<R>* sA = reinterpret_cast<cx<R>*>(smem_raw);   // A (MD x MD) then b (MD)
  const cx<R>* sb = sA + MD * MD;
  R* sq = reinterpret_cast<R*>(sA + MD * MD + MD);
  R* isq = sq + (kMaxCut + 4);
  int* spn = reinterpret_cast<int*>(isq + (kMaxCut + 4));
  const int pnw = P.pnw;
  for (int i = threadIdx.x; i < (MD + 1) * pnw; i += blockDim.x) spn[i] = P.pn[i];
  for (int v = threadIdx.x; v < kMaxCut + 4; v += blockDim.x) {
    sq[v] = sqrt(R(v));
    isq[v] = v ? R(1) / sqrt(R(v)) : R(0);
  }
  for (int i = threadIdx.x; i < MD * MD + MD; i += blockDim.x) sA[i] = ld(Ak + i);
  __syncthreads();
  const int stride = gridDim.x * blockDim.x;
  if (zlevel >= 0) {
    cx<R>* z = f0 + P.lvl[zlevel];
    const int nz = (int)(P.lvl[zlevel + 1] - P.lvl[zlevel]);
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nz; r += stride) st(z + r, czero<R>());
  }
  if (S < 1) return;
  cx<R>* cur = f0 + P.lvl[S];
  const cx<R>* lv1 = f0 + P.lvl[S - 1];
  const cx<R>* lv2 = S >= 2 ? f0 + P.lvl[S - 2] : f0;
  const int n = (int)(P.lvl[S + 1] - P.lvl[S]);
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    int m[MD], s[MD + 1], rdn[MD], rup[MD];
    unrank<MD>(spn, pnw, P.CD, S, r, m, s);
    neighbour_ranks<MD>(spn, pnw, s, rdn, rup);
    // first mode with a photon: its index, the parent's rank and n_i
    // (selected with constant indices)
    int i = 0, rp = 0, ni = 1;
    bool found = false;
#pragma unroll
    for (int d = 0; d < MD; ++d)
      if (!found && m[d] > 0) {
        found = true;
        i = d;
        rp = rdn[d];
        ni = m[d];
      }
    // partial sums of the parent p = m - 1_i, then its neighbours at S - 2
    int sp[MD + 1], pdn[MD], pup[MD];
#pragma unroll
    for (int d = 0; d <= MD; ++d) sp[d] = s[d] - (d <= i ? 1 : 0);
    sp[MD] = 0;
    cx<R> acc = czero<R>();
    if (!BZ) cfma(acc, sb[i], ld(lv1 + rp));
    if (S >= 2) {
      neighbour_ranks<MD>(spn, pnw, sp, pdn, pup);
#pragma unroll
      for (int l = 0; l < MD; ++l) {
        const int pl = m[l] - (l == i ? 1 : 0);
        if (pl > 0) cfma(acc, sA[i * MD + l], cscale(ld(lv2 + pdn[l]), sq[pl]));
      }
    }
    st(cur + r, cscale(acc, isq[ni]));
  }
}

// ---------------------------------------------------------------------------
// Reverse mode.  The local gradients of Sec. 2.5 (the solutions of its
// tangent recurrences for b and A) have closed forms in the amplitudes:
//   d psi_k / d b_i   = sqrt(k_i) psi_{k - 1_i},
//   d psi_k / d A_il  = 1/2 sqrt(k_i (k_l - [i = l])) psi_{k - 1_i - 1_l},
//   d psi_k / d c     = psi_k / c,
// and every shifted amplitude lies inside the box, so the cotangents
//   bbar_i = sum_k g_k conj(d psi_k / d b_i)   (g = dL/dpsi^*, Eqs. dL_dB, dL_dA)
// are weighted dot products of g with shifted copies of psi.  One launch
// accumulates up to kVjpGroup of them; each thread sums its indices in
// order, the workgroup folds its threads in a fixed tree into its slot, and
// the final kernel adds the slots in order (bitwise reproducible).
// ---------------------------------------------------------------------------
constexpr int kVjpTerms = kMaxD + kMaxD * (kMaxD + 1) / 2 + 1;   // bbar, Abar (i <= l), c

// The terms; mode i of term t has C-order stride si[t] and cutoff ci[t] (the
// same for l), with their reciprocals for the exact double-reciprocal digit
// split.
struct StateVjpTerms {
  int n;                    // terms (ncol)
  int col[kVjpTerms];       // output column of each term
  int kind[kVjpTerms];      // 0: bbar_i, 1: Abar_il (i < l), 2: Abar_ii, 3: sum g conj(psi)
  int si[kVjpTerms], ci[kVjpTerms], sl[kVjpTerms], cl[kVjpTerms];
  double inv_si[kVjpTerms], inv_ci[kVjpTerms], inv_sl[kVjpTerms], inv_cl[kVjpTerms];
};

// Digit (x / stride) mod C of a C-order index x < 2^31: (x + 1/2) / stride
// lies at least 1 / (2 stride) from an integer and the rounded product is off
// by less than (x / stride) 2^-51, so truncation is exact (and so for the mod).
__device__ __forceinline__ int cdigit(int x, int stride, int c, double inv_stride, double inv_c) {
  const int q = (int)((x + 0.5) * inv_stride);
  return q - c * (int)((q + 0.5) * inv_c);
}

// One workgroup per (chunk of `len` consecutive indices, term): the term is
// uniform, so each lane keeps one accumulator, the g and shifted psi reads
// of a wavefront are consecutive addresses, and the term's workgroups of one
// chunk run together (term fastest in the grid) and share the chunk's g in
// L2.  Each lane sums its indices in order, the workgroup folds its lanes in
// a fixed tree into slot (chunk, column); the final kernel adds the slots of
// a column in order (bitwise reproducible).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_state_vjp_terms(const cx<R>* __restrict__ psi,
                                                              const cx<R>* __restrict__ g, int total, int len,
                                                              StateVjpTerms T, double2* __restrict__ slots) {
  __shared__ double2 red[kThreads];
  __shared__ double sq[kMaxCut + 1];   // sqrt(0..64)
  for (int v = threadIdx.x; v <= kMaxCut; v += blockDim.x) sq[v] = sqrt((double)v);
  __syncthreads();
  const int term = (int)(blockIdx.x % (unsigned)T.n), chunk = (int)(blockIdx.x / (unsigned)T.n);
  const int kind = T.kind[term];
  const int si = T.si[term], ci = T.ci[term], sl = T.sl[term], cl = T.cl[term];
  const double isi = T.inv_si[term], ici = T.inv_ci[term], isl = T.inv_sl[term], icl = T.inv_cl[term];
  const int shift = kind == 0 ? si : kind == 1 ? si + sl : kind == 2 ? 2 * si : 0;
  const int x0 = chunk * len, x1 = min(total, x0 + len);
  double ax = 0.0, ay = 0.0;
  for (int x = x0 + threadIdx.x; x < x1; x += blockDim.x) {
    double w = 1.0;
    if (kind != 3) {
      const int ki = cdigit(x, si, ci, isi, ici);
      if (kind == 0) {
        w = sq[ki];
      } else if (kind == 1) {
        w = 0.5 * sq[ki] * sq[cdigit(x, sl, cl, isl, icl)];
      } else {
        w = ki >= 2 ? 0.5 * sq[ki] * sq[ki - 1] : 0.0;
      }
    }
    if (w != 0.0) {   // else the shifted amplitude is outside the box
      const cx<R> gv = ld(g + x), pv = ld(psi + (x - shift));
      // g * conj(w psi_y)
      const double px = w * (double)pv.x, py = w * (double)pv.y;
      ax += (double)gv.x * px + (double)gv.y * py;
      ay += (double)gv.y * px - (double)gv.x * py;
    }
  }
  red[threadIdx.x] = make_double2(ax, ay);
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[threadIdx.x].x += red[threadIdx.x + w].x;
      red[threadIdx.x].y += red[threadIdx.x + w].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) slots[(size_t)chunk * T.n + T.col[term]] = red[0];
}

// One workgroup per caller entry of dA (M x M), db (M), dc: the slots of its
// column added in order (zero for modes with cutoff 1), Abar mirrored.
struct StateVjpMap {
  int M, MD, ncol, nslots;
  int mode[kMaxD];
};

template <typename R>
__global__ __launch_bounds__(kThreads) void k_state_vjp_final(StateVjpMap m, const double2* __restrict__ slots,
                                                              const cx<R>* __restrict__ c, cx<R>* dA, cx<R>* db,
                                                              cx<R>* dc) {
  __shared__ double2 red[kThreads];
  const int e = blockIdx.x, M = m.M, MD = m.MD;
  int col = -1;
  if (e < M * M) {
    int ki = -1, kl = -1;
    for (int d = 0; d < MD; ++d) {
      if (m.mode[d] == e / M) ki = d;
      if (m.mode[d] == e % M) kl = d;
    }
    if (ki >= 0 && kl >= 0) {
      const int a = min(ki, kl), bb = max(ki, kl);
      col = MD + a * MD - a * (a - 1) / 2 + (bb - a);   // columns: bbar (MD), then the upper triangle row by row
    }
  } else if (e < M * M + M) {
    for (int d = 0; d < MD; ++d)
      if (m.mode[d] == e - M * M) col = d;
  } else {
    col = m.ncol - 1;
  }
  double sx = 0.0, sy = 0.0;
  if (col >= 0)
    for (int s = threadIdx.x; s < m.nslots; s += blockDim.x) {
      sx += slots[(size_t)s * m.ncol + col].x;
      sy += slots[(size_t)s * m.ncol + col].y;
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
  double2 t = red[0];
  if (e < M * M) {
    st(dA + e, cmake<R>((R)t.x, (R)t.y));
  } else if (e < M * M + M) {
    st(db + (e - M * M), cmake<R>((R)t.x, (R)t.y));
  } else {
    // cbar = sum g conj(psi / c) = (sum g conj(psi)) / conj(c)
    const cx<R> cv = ld(c);
    const double cr = (double)cv.x, ci = (double)cv.y, n2 = cr * cr + ci * ci;
    st(dc, cmake<R>((R)((t.x * cr - t.y * ci) / n2), (R)((t.y * cr + t.x * ci) / n2)));
  }
}

// Forward mode: the tangent of psi along (dA, db, dc), from the same closed
// forms, one thread per amplitude:
//   dpsi_k = (dc / c) psi_k + sum_i db_i sqrt(k_i) psi_{k-1_i}
//          + sum_{i <= l} S_il w_il(k) psi_{k-1_i-1_l},
// S_il = dA_il + dA_li (i < l), dA_ii (i = l), w_il = 1/2 sqrt(k_i k_l) or
// 1/2 sqrt(k_i (k_i - 1)): the directional derivative for the symmetric part
// of dA, as A enters through (A + A^T)/2.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_state_jvp(DevPlan P, StateModes sm, int M, const cx<R>* __restrict__ psi,
                                                        const cx<R>* __restrict__ c, const cx<R>* __restrict__ tA,
                                                        const cx<R>* __restrict__ tb, const cx<R>* __restrict__ tc,
                                                        int total, cx<R>* __restrict__ dpsi) {
  __shared__ double2 sS[kMaxD * kMaxD];
  __shared__ double2 sB[kMaxD];
  __shared__ double sq[kMaxCut + 1];   // sqrt(0..64)
  const int MD = P.MD;
  for (int v = threadIdx.x; v <= kMaxCut; v += blockDim.x) sq[v] = sqrt((double)v);
  for (int e = threadIdx.x; e < MD * MD; e += blockDim.x) {
    const int i = e / MD, l = e % MD;
    const cx<R> a = ld(tA + (size_t)sm.mode[i] * M + sm.mode[l]);
    const cx<R> t = ld(tA + (size_t)sm.mode[l] * M + sm.mode[i]);
    sS[e] = i == l ? make_double2(a.x, a.y) : make_double2((double)a.x + t.x, (double)a.y + t.y);
  }
  for (int i = threadIdx.x; i < MD; i += blockDim.x) {
    const cx<R> v = ld(tb + sm.mode[i]);
    sB[i] = make_double2(v.x, v.y);
  }
  __syncthreads();
  // dc / c
  const cx<R> cv = ld(c), dv = ld(tc);
  const double n2 = (double)cv.x * cv.x + (double)cv.y * cv.y;
  const double rx = ((double)dv.x * cv.x + (double)dv.y * cv.y) / n2, ry = ((double)dv.y * cv.x - (double)dv.x * cv.y) / n2;
  int stride[kMaxD];
  {
    int s = 1;
    for (int d = MD - 1; d >= 0; --d) {
      stride[d] = s;
      s *= P.CD[d];
    }
  }
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < total; x += gridDim.x * blockDim.x) {
    int k[kMaxD];
    int rem = x;
    for (int d = MD - 1; d >= 0; --d) {
      const int q = (int)((rem + 0.5) * P.cinv[d]);
      k[d] = rem - q * P.CD[d];
      rem = q;
    }
    const cx<R> p0 = ld(psi + x);
    double ax = rx * p0.x - ry * p0.y, ay = rx * p0.y + ry * p0.x;
    for (int i = 0; i < MD; ++i) {
      if (k[i] < 1) continue;
      const cx<R> p1 = ld(psi + x - stride[i]);
      const double w = sq[k[i]];
      const double2 t = sB[i];
      ax += w * (t.x * p1.x - t.y * p1.y);
      ay += w * (t.x * p1.y + t.y * p1.x);
      for (int l = i; l < MD; ++l) {
        const int kl = k[l] - (l == i ? 1 : 0);
        if (kl < 1) continue;
        const cx<R> p2 = ld(psi + x - stride[i] - stride[l]);
        const double w2 = 0.5 * sq[k[i]] * sq[kl];
        const double2 S = sS[i * MD + l];
        ax += w2 * (S.x * p2.x - S.y * p2.y);
        ay += w2 * (S.x * p2.y + S.y * p2.x);
      }
    }
    st(dpsi + x, cmake<R>((R)ax, (R)ay));
  }
}

hipError_t run_state_jvp(const Plan& Pl, const void* c, const void* psi, const void* dA, const void* db, const void* dc,
                         void* dpsi, hipStream_t st) {
  StateModes sm;
  std::memset(&sm, 0, sizeof(sm));
  sm.MD = Pl.MD;
  for (int k = 0; k < Pl.MD; ++k) sm.mode[k] = Pl.dmodes[k];
  const DevPlan P = make_devplan(Pl, true);
  const int total = (int)Pl.nodes_total;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + kThreads - 1) / kThreads, 65536));
  KTimer kt(Pl, KK_FWD_LEVEL, st);
  if (Pl.dt == FD_C64)
    hipLaunchKernelGGL((k_state_jvp<float>), dim3(grid), dim3(kThreads), 0, st, P, sm, Pl.M,
                       static_cast<const cx<float>*>(psi), static_cast<const cx<float>*>(c),
                       static_cast<const cx<float>*>(dA), static_cast<const cx<float>*>(db),
                       static_cast<const cx<float>*>(dc), total, static_cast<cx<float>*>(dpsi));
  else
    hipLaunchKernelGGL((k_state_jvp<double>), dim3(grid), dim3(kThreads), 0, st, P, sm, Pl.M,
                       static_cast<const cx<double>*>(psi), static_cast<const cx<double>*>(c),
                       static_cast<const cx<double>*>(dA), static_cast<const cx<double>*>(db),
                       static_cast<const cx<double>*>(dc), total, static_cast<cx<double>*>(dpsi));
  return hipGetLastError();
}

template <typename R>
static hipError_t run_state_vjp_t(const Plan& Pl, const void* c, const void* psi, const void* g, void* dA, void* db,
                                  void* dc, void* ws, hipStream_t st) {
  const int MD = Pl.MD, ncol = MD + MD * (MD + 1) / 2 + 1;
  const int total = (int)Pl.nodes_total;
  double2* slots = static_cast<double2*>(ws);
  // chunks of whole wavefront multiples, at most kVjpSlots of them
  int len = 16 * kThreads;
  while ((int64_t)(total + len - 1) / len > kVjpSlots) len *= 2;
  const int nchunks = std::max(1, (total + len - 1) / len);
  // the terms: bbar_i (col i), Abar_il for i <= l (col MD + upper-triangle index), sum g conj(psi) (last col)
  StateVjpTerms T;
  std::memset(&T, 0, sizeof(T));
  std::vector<int> cstride(MD > 0 ? MD : 1, 1);
  for (int d = MD - 2; d >= 0; --d) cstride[d] = cstride[d + 1] * Pl.CD[d + 1];
  auto add = [&](int col, int kind, int i, int l) {
    const int n = T.n++;
    T.col[n] = col;
    T.kind[n] = kind;
    if (kind != 3) {
      T.si[n] = cstride[i];
      T.ci[n] = Pl.CD[i];
      T.sl[n] = cstride[l];
      T.cl[n] = Pl.CD[l];
      T.inv_si[n] = 1.0 / cstride[i];
      T.inv_ci[n] = 1.0 / Pl.CD[i];
      T.inv_sl[n] = 1.0 / cstride[l];
      T.inv_cl[n] = 1.0 / Pl.CD[l];
    }
  };
  for (int i = 0; i < MD; ++i) add(i, 0, i, i);
  for (int a = 0; a < MD; ++a)
    for (int bb = a; bb < MD; ++bb) add(MD + a * MD - a * (a - 1) / 2 + (bb - a), a == bb ? 2 : 1, a, bb);
  add(ncol - 1, 3, 0, 0);
  {
    KTimer kt(Pl, KK_VJP_LEVEL, st);
    hipLaunchKernelGGL((k_state_vjp_terms<R>), dim3((unsigned)(nchunks * T.n)), dim3(kThreads), 0, st,
                       static_cast<const cx<R>*>(psi), static_cast<const cx<R>*>(g), total, len, T, slots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  StateVjpMap m;
  std::memset(&m, 0, sizeof(m));
  m.M = Pl.M;
  m.MD = MD;
  m.ncol = ncol;
  m.nslots = nchunks;
  for (int d = 0; d < MD; ++d) m.mode[d] = Pl.dmodes[d];
  KTimer kt(Pl, KK_VJP_FINAL, st);
  hipLaunchKernelGGL((k_state_vjp_final<R>), dim3(Pl.M * Pl.M + Pl.M + 1), dim3(kThreads), 0, st, m, slots,
                     static_cast<const cx<R>*>(c), static_cast<cx<R>*>(dA), static_cast<cx<R>*>(db),
                     static_cast<cx<R>*>(dc));
  return hipGetLastError();
}

hipError_t run_state_vjp(const Plan& Pl, const void* c, const void* psi, const void* g, void* dA, void* db, void* dc,
                         void* ws, hipStream_t st) {
  if (Pl.dt == FD_C64) return run_state_vjp_t<float>(Pl, c, psi, g, dA, db, dc, ws, st);
  return run_state_vjp_t<double>(Pl, c, psi, g, dA, db, dc, ws, st);
}

template <typename R>
static hipError_t run_state_fwd_t(const Plan& Pl, bool bz, const void* A, const void* b, const void* c, void* psi,
                                  void* ws, hipStream_t st) {
  const size_t eb = sizeof(cx<R>);
  cx<R>* f0 = static_cast<cx<R>*>(ws);
  cx<R>* Ak = reinterpret_cast<cx<R>*>(static_cast<char*>(ws) + (((size_t)Pl.nodes_total * eb + 255) & ~size_t(255)));
  StateModes sm;
  std::memset(&sm, 0, sizeof(sm));
  sm.MD = Pl.MD;
  for (int k = 0; k < Pl.MD; ++k) sm.mode[k] = Pl.dmodes[k];
  {
    KTimer kt(Pl, KK_PREP, st);
    hipLaunchKernelGGL((k_state_prep<R>), dim3(1), dim3(64), 0, st, Pl.M, sm, static_cast<const cx<R>*>(A),
                       static_cast<const cx<R>*>(b), static_cast<const cx<R>*>(c), Ak, f0, bz ? 1 : 0,
                       Pl.d_status);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const DevPlan P = make_devplan(Pl, !bz);
  const size_t shm = (size_t)(Pl.MD * Pl.MD + Pl.MD) * eb + 2 * (kMaxCut + 4) * sizeof(R) +
                     (size_t)(Pl.MD + 1) * (Pl.smax + 3) * sizeof(int);
  auto count = [&](int S) { return S >= 0 && S <= Pl.smax ? Pl.lvl[S + 1] - Pl.lvl[S] : int64_t(0); };
  auto launch = [&](int S, int zl) -> hipError_t {
    const int64_t work = std::max(count(S), count(zl));
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + kThreads - 1) / kThreads, 65536));
    KTimer kt(Pl, KK_FWD_LEVEL, st);
#define FD_STATE_LEVEL(MDV)                                                                                \
  case MDV:                                                                                                \
    if (bz)                                                                                                \
      hipLaunchKernelGGL((k_state_level<MDV, true, R>), dim3(grid), dim3(kThreads), shm, st, P, Ak, f0, S, zl); \
    else                                                                                                   \
      hipLaunchKernelGGL((k_state_level<MDV, false, R>), dim3(grid), dim3(kThreads), shm, st, P, Ak, f0, S, zl); \
    break;
    switch (Pl.MD) {
      FD_STATE_LEVEL(1)
      FD_STATE_LEVEL(2)
      FD_STATE_LEVEL(3)
      FD_STATE_LEVEL(4)
      FD_STATE_LEVEL(5)
      FD_STATE_LEVEL(6)
      FD_STATE_LEVEL(7)
      FD_STATE_LEVEL(8)
      default: return hipErrorInvalidValue;
    }
#undef FD_STATE_LEVEL
    return hipGetLastError();
  };
  for (int S = 1; S <= Pl.smax && Pl.MD > 0; ++S) {
    if (bz && (S & 1)) continue;   // odd level: cleared with the next even one
    if ((e = launch(S, bz ? S - 1 : -1)) != hipSuccess) return e;
  }
  if (bz && Pl.MD > 0 && (Pl.smax & 1))
    if ((e = launch(-1, Pl.smax)) != hipSuccess) return e;
  return launch_out_perm(Pl, f0, psi, st);
}

hipError_t run_state_fwd(const Plan& Pl, bool b_zero, const void* A, const void* b, const void* c, void* psi, void* ws,
                         hipStream_t st) {
  if (Pl.dt == FD_C64) return run_state_fwd_t<float>(Pl, b_zero, A, b, c, psi, ws, st);
  return run_state_fwd_t<double>(Pl, b_zero, A, b, c, psi, ws, st);
}

}  // namespace fd
