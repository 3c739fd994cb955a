/*
 * Seeded synthetic inputs for the source-to-waveform map.
 *
 * This module generates inputs only: subfault, seafloor-grid and observer
 * positions; time-domain elastic Green's-function blocks G[g][j][k]
 * (the entries of F_{G,k}, paper Sec. II-B1, eq. 1); time-domain
 * acoustic-gravity response blocks F[g][o][k] (the entries of F_{q,k},
 * Sec. II-B2, eq. 2); slip-rate histories s[j][n]; observation noise.
 * It holds none of the method's arithmetic (no convolution, no transform),
 * and serves both the FP64 oracle and the GPU library's callers.
 *
 * Every value is a pure function of (seed, tag, i, j, c) through a
 * counter-based generator, so any chunk of grid rows, any subset of
 * columns and any single rupture regenerate bit-identically, in any order
 * and on any number of threads.
 *
 * Counter-based generator: the SplitMix64 output function (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014)
 * applied to a chained key; uniforms take the top 53 bits; normals use the
 * Box-Muller transform (Box and Muller, Ann. Math. Statist. 1958).
 *
 * The paper's inputs (FakeQuakes ruptures, FK Green's functions, adjoint
 * acoustic-gravity responses) are not available; these stand in for them
 * with the paper's shapes (Sec. III-C, Table II): a damped sinusoid per
 * source/receiver pair with spatial decay and a travel-time onset, and
 * triangle slip-rate pulses that start at a rupture-front arrival time.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#define S2W_SYNTH_PI 3.14159265358979323846

enum {
  TAG_POS_SUB = 1, TAG_POS_GRID = 2, TAG_POS_OBS = 3,
  TAG_G_PAR = 4, TAG_F_PAR = 5, TAG_SLIP = 6,
  TAG_DENSE_G = 7, TAG_DENSE_F = 8, TAG_DENSE_S = 9,
  TAG_NOISE = 10, TAG_VEC = 11
};

/* Kinds of operator: 0 = damped-sinusoid physical form, 1 = dense iid N(0,1). */
typedef struct {
  int64_t nsub, ngrid, nobs, nt;
  double dt;          /* seconds per step */
  uint64_t seed;       /* positions and operators */
  uint64_t slip_seed;  /* slip-rate draws */
  int32_t op_kind;    /* 0 physical form, 1 dense iid N(0,1) */
  int32_t slip_mode;  /* 0 all active, 1 rupture length U(len_lo,len_hi), 2 K nearest U{k_lo..nsub}, 3 dense iid N(0,1) */
  double box_x, box_y;    /* km */
  double v_g, v_f;        /* travel speeds, km/s, of the elastic and acoustic responses */
  double decay_km;        /* spatial decay length, km */
  double tau_lo, tau_hi;  /* s */
  double f_lo, f_hi;      /* Hz */
  double v_rup;           /* rupture-front speed, km/s */
  double w_lo, w_hi;      /* triangle pulse width range, s (equal = fixed) */
  double len_lo, len_hi;  /* rupture length range, km (slip_mode 1) */
  int64_t k_lo;           /* minimum active count (slip_mode 2) */
} s2w_synth_cfg;

static inline uint64_t sm64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static inline uint64_t key5(uint64_t seed, uint64_t tag, uint64_t i, uint64_t j, uint64_t c) {
  uint64_t h = sm64(seed);
  h = sm64(h ^ tag);
  h = sm64(h ^ i);
  h = sm64(h ^ j);
  return sm64(h ^ c);
}

/* uniform in the open interval (0,1) */
static inline double u01(uint64_t h) { return ((double)(h >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

static inline double normal(uint64_t seed, uint64_t tag, uint64_t i, uint64_t j, uint64_t c) {
  /* Box-Muller from two independent keyed uniforms */
  double a = u01(key5(seed, tag, i, j, 2 * c));
  double b = u01(key5(seed, tag, i, j, 2 * c + 1));
  return sqrt(-2.0 * log(a)) * cos(2.0 * S2W_SYNTH_PI * b);
}

double s2w_synth_uniform(uint64_t seed, uint64_t tag, uint64_t i, uint64_t j, uint64_t c) {
  return u01(key5(seed, tag, i, j, c));
}
double s2w_synth_normal(uint64_t seed, uint64_t tag, uint64_t i, uint64_t j, uint64_t c) {
  return normal(seed, tag, i, j, c);
}

/* kind: 0 subfaults, 1 grid points, 2 observers; writes n (x,y) pairs in km */
void s2w_synth_positions(const s2w_synth_cfg* c, int32_t kind, int64_t i0, int64_t n, double* xy) {
  uint64_t tag = kind == 0 ? TAG_POS_SUB : (kind == 1 ? TAG_POS_GRID : TAG_POS_OBS);
  for (int64_t i = 0; i < n; i++) {
    xy[2 * i + 0] = c->box_x * u01(key5(c->seed, tag, (uint64_t)(i0 + i), 0, 0));
    xy[2 * i + 1] = c->box_y * u01(key5(c->seed, tag, (uint64_t)(i0 + i), 0, 1));
  }
}

static inline double pos1(const s2w_synth_cfg* c, uint64_t tag, int64_t i, int axis) {
  return (axis ? c->box_y : c->box_x) * u01(key5(c->seed, tag, (uint64_t)i, 0, (uint64_t)axis));
}

/*
 * One damped-sinusoid response series of length nt for a (receiver, source) pair:
 * A exp(-dist/decay) exp(-t/tau) sin(2 pi f t + phi) for t >= dist/speed, zero before.
 * Past the onset sample the exponential and the sinusoid advance by a
 * constant ratio and a constant rotation per step (exact in real arithmetic;
 * in double precision the drift over a few hundred steps is ~1e-14 relative,
 * far below the float32 rounding of the stored value).
 */
static void pair_series(const s2w_synth_cfg* c, uint64_t ptag, int64_t a, int64_t b, double dist,
                        double speed, float* out) {
  const int64_t nt = c->nt;
  const double dt = c->dt;
  double A = normal(c->seed, ptag, (uint64_t)a, (uint64_t)b, 0);
  double tau = c->tau_lo + (c->tau_hi - c->tau_lo) * u01(key5(c->seed, ptag, (uint64_t)a, (uint64_t)b, 2));
  double f = c->f_lo + (c->f_hi - c->f_lo) * u01(key5(c->seed, ptag, (uint64_t)a, (uint64_t)b, 3));
  double phi = 2.0 * S2W_SYNTH_PI * u01(key5(c->seed, ptag, (uint64_t)a, (uint64_t)b, 4));
  double amp = A * exp(-dist / c->decay_km);
  double t0 = dist / speed;
  int64_t k = 0;
  for (; k < nt && (double)k * dt < t0; k++) out[k] = 0.0f;
  if (k == nt) return;
  double t = (double)k * dt;
  double e = amp * exp(-t / tau), q = exp(-dt / tau);
  double w = 2.0 * S2W_SYNTH_PI * f;
  double sn = sin(w * t + phi), cs = cos(w * t + phi);
  double rs = sin(w * dt), rc = cos(w * dt);
  for (; k < nt; k++) {
    out[k] = (float)(e * sn);
    double sn2 = sn * rc + cs * rs;
    double cs2 = cs * rc - sn * rs;
    sn = sn2; cs = cs2;
    e *= q;
  }
}

/*
 * Elastic blocks for grid rows [row0, row0+nrows) and the subfault columns
 * cols[0..ncols) (cols == NULL means all nsub in order):
 * out[r][q][k] = [F_{G,k}]_{row0+r, cols[q]}.
 */
void s2w_synth_G(const s2w_synth_cfg* c, int64_t row0, int64_t nrows, const int64_t* cols, int64_t ncols,
                 float* out) {
  const int64_t nt = c->nt;
  if (!cols) ncols = c->nsub;
  double* sxy = (double*)malloc(sizeof(double) * 2 * (size_t)(ncols > 0 ? ncols : 1));
  for (int64_t q = 0; q < ncols; q++) {
    int64_t j = cols ? cols[q] : q;
    sxy[2 * q] = pos1(c, TAG_POS_SUB, j, 0);
    sxy[2 * q + 1] = pos1(c, TAG_POS_SUB, j, 1);
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t r = 0; r < nrows; r++) {
    int64_t g = row0 + r;
    double gx = pos1(c, TAG_POS_GRID, g, 0), gy = pos1(c, TAG_POS_GRID, g, 1);
    for (int64_t q = 0; q < ncols; q++) {
      int64_t j = cols ? cols[q] : q;
      float* o = out + (r * ncols + q) * nt;
      if (c->op_kind == 1) {
        for (int64_t k = 0; k < nt; k++) o[k] = (float)normal(c->seed, TAG_DENSE_G, (uint64_t)g, (uint64_t)j, (uint64_t)k);
      } else {
        double dx = gx - sxy[2 * q], dy = gy - sxy[2 * q + 1];
        pair_series(c, TAG_G_PAR, g, j, sqrt(dx * dx + dy * dy), c->v_g, o);
      }
    }
  }
  free(sxy);
}

/* Acoustic-gravity blocks: out[r][o][k] = [F_{q,k}]_{o, row0+r}. */
void s2w_synth_F(const s2w_synth_cfg* c, int64_t row0, int64_t nrows, float* out) {
  const int64_t nt = c->nt, nobs = c->nobs;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t r = 0; r < nrows; r++) {
    int64_t g = row0 + r;
    double gx = pos1(c, TAG_POS_GRID, g, 0), gy = pos1(c, TAG_POS_GRID, g, 1);
    for (int64_t o = 0; o < nobs; o++) {
      float* p = out + (r * nobs + o) * nt;
      if (c->op_kind == 1) {
        for (int64_t k = 0; k < nt; k++) p[k] = (float)normal(c->seed, TAG_DENSE_F, (uint64_t)g, (uint64_t)o, (uint64_t)k);
      } else {
        double dx = gx - pos1(c, TAG_POS_OBS, o, 0), dy = gy - pos1(c, TAG_POS_OBS, o, 1);
        pair_series(c, TAG_F_PAR, g, o, sqrt(dx * dx + dy * dy), c->v_f, p);
      }
    }
  }
}

typedef struct { double d; int64_t j; } dist_idx;
static int cmp_dist(const void* a, const void* b) {
  const dist_idx* x = (const dist_idx*)a; const dist_idx* y = (const dist_idx*)b;
  if (x->d < y->d) return -1;
  if (x->d > y->d) return 1;
  return (x->j < y->j) ? -1 : (x->j > y->j);
}

/*
 * Slip-rate history of rupture number `rup`: out[j][n], j < nsub, n < nt.
 * Triangle pulse of width W starting at the rupture-front arrival
 * |x_j - x_h| / v_rup, peak a_j ~ U(0,1) at onset + W/2; inactive subfaults are zero.
 * info (may be NULL) receives {hypocentre, active count, W, length-or-K}.
 */
void s2w_synth_slip(const s2w_synth_cfg* c, int64_t rup, float* out, double* info) {
  const int64_t nsub = c->nsub, nt = c->nt;
  const uint64_t sd = c->slip_seed;
  if (c->slip_mode == 3) {
    for (int64_t j = 0; j < nsub; j++)
      for (int64_t n = 0; n < nt; n++) out[j * nt + n] = (float)normal(sd, TAG_DENSE_S, (uint64_t)rup, (uint64_t)j, (uint64_t)n);
    if (info) { info[0] = -1; info[1] = (double)nsub; info[2] = 0; info[3] = 0; }
    return;
  }
  int64_t h = (int64_t)(u01(key5(sd, TAG_SLIP, (uint64_t)rup, 0, 0)) * (double)nsub);
  if (h >= nsub) h = nsub - 1;
  double W = c->w_lo + (c->w_hi - c->w_lo) * u01(key5(sd, TAG_SLIP, (uint64_t)rup, 0, 1));
  double hx = pos1(c, TAG_POS_SUB, h, 0), hy = pos1(c, TAG_POS_SUB, h, 1);
  dist_idx* di = (dist_idx*)malloc(sizeof(dist_idx) * (size_t)nsub);
  for (int64_t j = 0; j < nsub; j++) {
    double dx = pos1(c, TAG_POS_SUB, j, 0) - hx, dy = pos1(c, TAG_POS_SUB, j, 1) - hy;
    di[j].d = sqrt(dx * dx + dy * dy);
    di[j].j = j;
  }
  unsigned char* act = (unsigned char*)calloc((size_t)nsub, 1);
  double extent = 0;
  int64_t nact = 0;
  if (c->slip_mode == 0) {
    for (int64_t j = 0; j < nsub; j++) act[j] = 1;
    nact = nsub;
  } else if (c->slip_mode == 1) {
    extent = c->len_lo + (c->len_hi - c->len_lo) * u01(key5(sd, TAG_SLIP, (uint64_t)rup, 0, 2));
    for (int64_t j = 0; j < nsub; j++)
      if (di[j].d <= 0.5 * extent) { act[j] = 1; nact++; }
  } else {
    int64_t klo = c->k_lo < nsub ? c->k_lo : nsub;
    int64_t K = klo + (int64_t)(u01(key5(sd, TAG_SLIP, (uint64_t)rup, 0, 3)) * (double)(nsub - klo + 1));
    if (K > nsub) K = nsub;
    dist_idx* srt = (dist_idx*)malloc(sizeof(dist_idx) * (size_t)nsub);
    memcpy(srt, di, sizeof(dist_idx) * (size_t)nsub);
    qsort(srt, (size_t)nsub, sizeof(dist_idx), cmp_dist);
    for (int64_t q = 0; q < K; q++) act[srt[q].j] = 1;
    free(srt);
    nact = K;
    extent = (double)K;
  }
  for (int64_t j = 0; j < nsub; j++) {
    float* o = out + j * nt;
    if (!act[j]) { for (int64_t n = 0; n < nt; n++) o[n] = 0.0f; continue; }
    double a = u01(key5(sd, TAG_SLIP, (uint64_t)rup, (uint64_t)(j + 1), 4));
    double onset = di[j].d / c->v_rup;
    double half = 0.5 * W;
    for (int64_t n = 0; n < nt; n++) {
      double t = (double)n * c->dt;
      double tri = 1.0 - fabs(t - onset - half) / half;
      o[n] = tri > 0.0 ? (float)(a * tri) : 0.0f;
    }
  }
  if (info) { info[0] = (double)h; info[1] = (double)nact; info[2] = W; info[3] = extent; }
  free(act);
  free(di);
}

/* iid N(0,1) test vector of length n under (tag-stream, index). */
void s2w_synth_normals(uint64_t seed, uint64_t stream, int64_t idx, int64_t n, double* out) {
  for (int64_t i = 0; i < n; i++) out[i] = normal(seed, TAG_VEC, stream, (uint64_t)idx, (uint64_t)i);
}

/* Observation noise: out[i] = N(0,1) for the hidden-rupture data, i < n. */
void s2w_synth_noise(uint64_t seed, int64_t n, double* out) {
  for (int64_t i = 0; i < n; i++) out[i] = normal(seed, TAG_NOISE, 0, 0, (uint64_t)i);
}
