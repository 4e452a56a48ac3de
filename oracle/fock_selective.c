/*
 * Selective Fock amplitudes on the CPU, by the pivot schedules of the paper
 * applied as printed -- TEST INFRASTRUCTURE ONLY (called from tests/ and the
 * CPU-baseline leg of bench.py through oracle/selective.py; it shares no code
 * with the GPU library).
 *
 * Amplitudes G_k of the 2M-index k = [ket_1, bra_1, ket_2, bra_2, ...]
 * (Sec. 2.1) are kept in a hash map keyed by k.  Applying a pivot p writes
 * G_{p+1_i} for the increments i of its write set by Eq. recrel:
 *
 *     sqrt(p_i + 1) G_{p+1_i} = b_i G_p + sum_l A_il sqrt(p_l) G_{p-1_l},
 *
 * reading G_p and G_{p-1_l} from the map; a read of an amplitude that no
 * earlier pivot wrote is reported as an error (the schedule would not be
 * self-sufficient, Sec. 3.1).  A target written a second time must agree
 * with the first value to 1e-9 relative (any route gives the same
 * amplitude), else an error is reported.
 *
 * Schedules:
 *   Algorithm 1 (every mode detected): for w = 0 .. sum C_j - 1, the diagonal
 *     pivots d = [a,a,b,b,...] with a+b+... = w and a < C_1 - 1, then the
 *     off-diagonal pivots d + 1_ket(j) for every j whose earlier modes are 0
 *     in d and whose d_j < C_j - 1; every pivot writes all its increments
 *     inside the box.
 *   Algorithm 2 (undetected modes U present; the paper's one-mode version
 *     extended to several undetected modes): step 1 applies every entry of
 *     the undetected block at zero detections in order of increasing weight,
 *     writing only undetected increments; step 2 is Algorithm 1 over the
 *     detected modes, each of its pivots applied as the whole block of
 *     undetected entries (in order of increasing weight) and writing only
 *     detected increments.
 * Every weight level of pivots is independent (Sec. 2.2); the pivots of one
 * level are distributed over OpenMP threads when nthreads > 1.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXM 16
#define MAXP (2 * MAXM)

typedef double complex cplx;

/* ---- open-addressing hash map: multi-index key -> amplitude ---- */
typedef struct {
  uint64_t* keys; /* key + 1; 0 = empty */
  cplx* vals;
  uint64_t mask;
} amap;

static int map_init(amap* m, uint64_t want) {
  uint64_t cap = 1024;
  while (cap < 2 * want) cap <<= 1;
  m->keys = (uint64_t*)calloc(cap, sizeof(uint64_t));
  m->vals = (cplx*)malloc(cap * sizeof(cplx));
  m->mask = cap - 1;
  return m->keys && m->vals ? 0 : -1;
}

static void map_free(amap* m) {
  free(m->keys);
  free(m->vals);
}

static uint64_t hash64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}

/* slot of key k, or of the empty slot where it would go */
static uint64_t map_slot(const amap* m, uint64_t k) {
  uint64_t s = hash64(k) & m->mask;
  while (m->keys[s] && m->keys[s] != k + 1) s = (s + 1) & m->mask;
  return s;
}

static int map_get(const amap* m, uint64_t k, cplx* v) {
  const uint64_t s = map_slot(m, k);
  if (!m->keys[s]) return 0;
  *v = m->vals[s];
  return 1;
}

/* ---- problem ---- */
typedef struct {
  int M, P;                 /* modes, positions (2M) */
  int cut[MAXM];            /* cutoff per mode */
  int det[MAXM];            /* 1: detected */
  uint64_t stride[MAXP];    /* mixed-radix key strides over the box */
  const cplx* A;            /* P x P, interleaved positions, symmetric part */
  const cplx* b;            /* P */
  amap map;
  int64_t pivots;           /* pivots applied */
  int err;                  /* 1: a read before its write; 2: inconsistent double write; 3: out of memory */
} prob;

static uint64_t key_of(const prob* pr, const int* k) {
  uint64_t x = 0;
  for (int p = 0; p < pr->P; ++p) x += (uint64_t)k[p] * pr->stride[p];
  return x;
}

/* Applies pivot k, writing the increments i with wmask[i] set; the new
 * values are returned in (tk[n], tv[n]) so that pivots of one level can run
 * in parallel and be merged afterwards. */
static int apply_pivot(const prob* pr, const int* k, const int* wmask, uint64_t* tk, cplx* tv, int* err) {
  const int P = pr->P;
  cplx g = 0.0, rd[MAXP];
  const uint64_t key = key_of(pr, k);
  int need_g = 0;
  for (int i = 0; i < P; ++i)
    if (wmask[i] && pr->b[i] != 0.0) need_g = 1;
  if (need_g && !map_get(&pr->map, key, &g)) {
    *err = 1;
    return 0;
  }
  for (int l = 0; l < P; ++l) {
    rd[l] = 0.0;
    if (k[l] > 0 && !map_get(&pr->map, key - pr->stride[l], &rd[l])) {
      *err = 1;
      return 0;
    }
  }
  int n = 0;
  for (int i = 0; i < P; ++i) {
    if (!wmask[i] || k[i] + 1 >= pr->cut[i / 2]) continue;
    cplx acc = pr->b[i] * g;
    for (int l = 0; l < P; ++l)
      if (k[l] > 0) acc += pr->A[(size_t)i * P + l] * sqrt((double)k[l]) * rd[l];
    tk[n] = key + pr->stride[i];
    tv[n] = acc / sqrt((double)(k[i] + 1));
    ++n;
  }
  return n;
}

/* Applies a list of pivots (one weight level: independent), then stores
 * their writes in list order. */
static void apply_level(prob* pr, const int* ks, int64_t npiv, const int* wmask, int nthreads) {
  const int P = pr->P;
  uint64_t* tk = (uint64_t*)malloc((size_t)(npiv > 0 ? npiv : 1) * P * sizeof(uint64_t));
  cplx* tv = (cplx*)malloc((size_t)(npiv > 0 ? npiv : 1) * P * sizeof(cplx));
  int* tn = (int*)calloc((size_t)(npiv > 0 ? npiv : 1), sizeof(int));
  if (!tk || !tv || !tn) {
    pr->err = 3;
    free(tk);
    free(tv);
    free(tn);
    return;
  }
  int err = 0;
#pragma omp parallel for num_threads(nthreads) schedule(static) reduction(| : err) if (nthreads > 1)
  for (int64_t q = 0; q < npiv; ++q) {
    int e = 0;
    tn[q] = apply_pivot(pr, ks + (size_t)q * P, wmask, tk + (size_t)q * P, tv + (size_t)q * P, &e);
    err |= e;
  }
  if (err) pr->err = err;
  for (int64_t q = 0; q < npiv && !pr->err; ++q)
    for (int j = 0; j < tn[q]; ++j) {
      const uint64_t s = map_slot(&pr->map, tk[(size_t)q * P + j]);
      const cplx v = tv[(size_t)q * P + j];
      if (pr->map.keys[s]) {
        const cplx old = pr->map.vals[s];
        if (cabs(v - old) > 1e-9 * fmax(cabs(old), 1e-300)) pr->err = 2;
      } else {
        pr->map.keys[s] = tk[(size_t)q * P + j] + 1;
        pr->map.vals[s] = v;
      }
    }
  pr->pivots += npiv;
  free(tk);
  free(tv);
  free(tn);
}

/* All points n of the box prod cuts[j] (nd modes) with sum w, in C order. */
static int64_t points_with_sum(int nd, const int* cuts, int w, int** out) {
  int64_t total = 1;
  for (int j = 0; j < nd; ++j) total *= cuts[j];
  int64_t cnt = 0, capn = 64;
  int* buf = (int*)malloc((size_t)capn * (nd > 0 ? nd : 1) * sizeof(int));
  int v[MAXM];
  for (int64_t x = 0; x < total; ++x) {
    int64_t r = x;
    int s = 0;
    for (int j = nd - 1; j >= 0; --j) {
      v[j] = (int)(r % cuts[j]);
      r /= cuts[j];
      s += v[j];
    }
    if (s != w) continue;
    if (cnt == capn) {
      capn *= 2;
      buf = (int*)realloc(buf, (size_t)capn * nd * sizeof(int));
    }
    memcpy(buf + (size_t)cnt * nd, v, (size_t)nd * sizeof(int));
    ++cnt;
  }
  *out = buf;
  return cnt;
}

/*
 * fd_oracle_selective -- the selected amplitudes rho[k_U.., l_U.., n_D..]
 * (C order; undetected kets, then undetected bras, then detected modes) of
 * the triple (A, b, c) given in interleaved positions (A: P x P with
 * P = 2M, its symmetric part is used; b: P; complex as (re, im) doubles).
 *   cut, det   per mode: cutoff >= 1, 1 if detected
 *   out        prod_U C^2 prod_D C complex outputs
 *   pivots     receives the number of pivots applied (NULL allowed)
 * Returns 0, or 1 (a read before its write), 2 (two writes disagree),
 * 3 (out of memory), 4 (bad arguments).
 */
int fd_oracle_selective(int M, const int* cut, const int* det, const double* A_ri, const double* b_ri,
                        const double* c_ri, double* out, int64_t* pivots, int nthreads) {
  if (M < 1 || M > MAXM) return 4;
  prob pr;
  memset(&pr, 0, sizeof(pr));
  pr.M = M;
  pr.P = 2 * M;
  const int P = pr.P;
  double box = 1.0;
  for (int j = 0; j < M; ++j) {
    if (cut[j] < 1 || cut[j] > 64) return 4;
    pr.cut[j] = cut[j];
    pr.det[j] = det[j] ? 1 : 0;
    box *= (double)cut[j] * cut[j];
  }
  if (box >= 9.0e18) return 4;
  {
    uint64_t s = 1;
    for (int p = P - 1; p >= 0; --p) {
      pr.stride[p] = s;
      s *= (uint64_t)cut[p / 2];
    }
  }
  cplx* As = (cplx*)malloc((size_t)P * P * sizeof(cplx));
  cplx* bs = (cplx*)malloc((size_t)P * sizeof(cplx));
  for (int i = 0; i < P; ++i) {
    bs[i] = b_ri[2 * i] + I * b_ri[2 * i + 1];
    for (int l = 0; l < P; ++l) {
      const cplx a = A_ri[2 * ((size_t)i * P + l)] + I * A_ri[2 * ((size_t)i * P + l) + 1];
      const cplx t = A_ri[2 * ((size_t)l * P + i)] + I * A_ri[2 * ((size_t)l * P + i) + 1];
      As[(size_t)i * P + l] = 0.5 * (a + t);
    }
  }
  pr.A = As;
  pr.b = bs;
  /* modes: undetected U and detected D, in caller order */
  int U[MAXM], D[MAXM], nu = 0, nd = 0;
  for (int j = 0; j < M; ++j) {
    if (pr.det[j])
      D[nd++] = j;
    else
      U[nu++] = j;
  }
  int64_t blk = 1, dbox = 1;
  for (int u = 0; u < nu; ++u) blk *= (int64_t)cut[U[u]] * cut[U[u]];
  for (int d = 0; d < nd; ++d) dbox *= cut[D[d]];
  /* expected entries: every pivot writes at most P amplitudes */
  if (map_init(&pr.map, (uint64_t)(blk * dbox * 2 * (P + 1) + 64)) != 0) {
    free(As);
    free(bs);
    return 3;
  }
  {
    const uint64_t s = map_slot(&pr.map, 0);
    pr.map.keys[s] = 1;
    pr.map.vals[s] = c_ri[0] + I * c_ri[1]; /* G_0 = c */
  }
  int wU[MAXP], wD[MAXP], wAll[MAXP];
  for (int p = 0; p < P; ++p) {
    wU[p] = !pr.det[p / 2];
    wD[p] = pr.det[p / 2];
    wAll[p] = 1;
  }
  /* the undetected block's entries by weight: 2 nu indices (kets, bras) */
  int bcut[MAXP];
  for (int u = 0; u < nu; ++u) bcut[u] = bcut[nu + u] = cut[U[u]];
  int bw = 0;
  for (int q = 0; q < 2 * nu; ++q) bw += bcut[q] - 1;
  int* kbuf = NULL;
  int64_t kcap = 0;
  /* step 1 (Algorithm 2 only): the block at zero detections, by weight */
  if (nu > 0) {
    for (int w = 0; w <= bw && !pr.err; ++w) {
      int* pts;
      const int64_t np = points_with_sum(2 * nu, bcut, w, &pts);
      if (np > kcap) {
        kcap = np;
        kbuf = (int*)realloc(kbuf, (size_t)kcap * P * sizeof(int));
      }
      for (int64_t x = 0; x < np; ++x) {
        int* k = kbuf + (size_t)x * P;
        memset(k, 0, (size_t)P * sizeof(int));
        for (int u = 0; u < nu; ++u) {
          k[2 * U[u]] = pts[(size_t)x * 2 * nu + u];
          k[2 * U[u] + 1] = pts[(size_t)x * 2 * nu + nu + u];
        }
      }
      apply_level(&pr, kbuf, np, wU, nthreads);
      free(pts);
    }
  }
  /* Algorithm 1 over the detected modes (step 2 of Algorithm 2): each
   * pivot is the block of undetected entries at that detected index */
  int dcut[MAXM];
  int wsum = 0;
  for (int d = 0; d < nd; ++d) {
    dcut[d] = cut[D[d]];
    wsum += dcut[d];
  }
  int* upts = NULL;
  int64_t nup = 0;
  {
    /* undetected entries in order of increasing weight */
    int64_t cap = blk > 0 ? blk : 1;
    upts = (int*)malloc((size_t)cap * (2 * nu > 0 ? 2 * nu : 1) * sizeof(int));
    for (int w = 0; w <= bw; ++w) {
      int* pts;
      const int64_t np = points_with_sum(2 * nu, bcut, w, &pts);
      memcpy(upts + (size_t)nup * 2 * nu, pts, (size_t)np * 2 * nu * sizeof(int));
      nup += np;
      free(pts);
    }
    if (nu == 0) nup = 1;
  }
  for (int w = 0; w < wsum && !pr.err; ++w) {
    int* dg;
    const int64_t ndg = points_with_sum(nd, dcut, w, &dg);
    /* diagonal pivots, then off-diagonal (bridge) pivots; each a block */
    for (int phase = 0; phase < 2 && !pr.err; ++phase) {
      int64_t np = 0;
      const int64_t most = ndg * nup * (phase ? nd : 1);
      if (most > kcap) {
        kcap = most;
        kbuf = (int*)realloc(kbuf, (size_t)kcap * P * sizeof(int));
      }
      for (int64_t x = 0; x < ndg; ++x) {
        const int* a = dg + (size_t)x * nd;
        for (int j = 0; j < (phase ? nd : 1); ++j) {
          if (!phase) {
            if (nd == 0 || a[0] >= dcut[0] - 1) continue; /* diag_1 < C_1 - 1 */
          } else {
            int zeros = 1;
            for (int q = 0; q < j; ++q) zeros = zeros && a[q] == 0; /* earlier modes 0 */
            if (!zeros || a[j] >= dcut[j] - 1) continue;
          }
          for (int64_t y = 0; y < nup; ++y) {
            int* k = kbuf + (size_t)np * P;
            memset(k, 0, (size_t)P * sizeof(int));
            for (int u = 0; u < nu; ++u) {
              k[2 * U[u]] = upts[(size_t)y * 2 * nu + u];
              k[2 * U[u] + 1] = upts[(size_t)y * 2 * nu + nu + u];
            }
            for (int d = 0; d < nd; ++d) k[2 * D[d]] = k[2 * D[d] + 1] = a[d];
            if (phase) k[2 * D[j]] += 1; /* diag + 1_ket(j) */
            ++np;
          }
        }
      }
      apply_level(&pr, kbuf, np, nu > 0 ? wD : wAll, nthreads);
    }
    free(dg);
  }
  /* outputs: rho[k_U.., l_U.., n_D..] in C order */
  int64_t nout = blk * dbox;
  for (int64_t x = 0; x < nout && !pr.err; ++x) {
    int k[MAXP];
    memset(k, 0, sizeof(k));
    int64_t r = x;
    for (int d = nd - 1; d >= 0; --d) {
      const int v = (int)(r % dcut[d]);
      r /= dcut[d];
      k[2 * D[d]] = k[2 * D[d] + 1] = v;
    }
    for (int u = nu - 1; u >= 0; --u) {
      k[2 * U[u] + 1] = (int)(r % cut[U[u]]);
      r /= cut[U[u]];
    }
    for (int u = nu - 1; u >= 0; --u) {
      k[2 * U[u]] = (int)(r % cut[U[u]]);
      r /= cut[U[u]];
    }
    cplx v;
    if (!map_get(&pr.map, key_of(&pr, k), &v)) {
      pr.err = 1;
      break;
    }
    out[2 * x] = creal(v);
    out[2 * x + 1] = cimag(v);
  }
  if (pivots) *pivots = pr.pivots;
  const int err = pr.err;
  map_free(&pr.map);
  free(kbuf);
  free(upts);
  free(As);
  free(bs);
  return err;
}
