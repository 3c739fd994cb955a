/*
 * FP64 CPU oracle for the source-to-waveform map -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the GPU library: no FFT, no
 * frequency domain, no blocking beyond the loops written here.  It evaluates
 * the paper's definitions directly in the time domain, in double precision:
 *
 *   elastic response, eq. (1):   m_n = sum_{k=0}^{n} F_{G,k} s_{n-k}
 *   temporal difference D_t:     v = D_t m, applied per seafloor point
 *                                (Sec. II-B2; read as the backward difference
 *                                v_n = (m_n - m_{n-1})/dt with m_{-1} = 0,
 *                                or as the identity when diff = 0)
 *   waveform response, eq. (2):  q_n = sum_{k=0}^{n} F_{q,k} v_{n-k}
 *
 * each convolution written in the channel form of eq. (4):
 * y_i[n] = sum_j sum_{k=0}^{n} f_ij[k] x_j[n-k].  Summed over the grid rows of
 * one share this is one rank's term of the distributed composition, eq. (3).
 *
 * The adjoint is the transpose of that real linear map (the block
 * lower-triangular Toeplitz operators of Sec. II-B3 transposed):
 *   w_g[n]  = sum_o sum_{k=0}^{Nt-1-n} f_{o,g}[k] r_o[n+k]
 *   w'_g[n] = (w_g[n] - w_g[n+1])/dt with w_g[Nt] = 0      (D_t transposed)
 *   gs_j[n] = sum_g sum_{k=0}^{Nt-1-n} g_{g,j}[k] w'_g[n+k]
 *
 * Layouts (row-major): G[g][j][k] = [F_{G,k}]_{g,j}, F[g][o][k] = [F_{q,k}]_{o,g},
 * s[b][j][n], y[b][o][n], r[b][o][n], gs[b][j][n].  The *_accum entry points
 * ADD the contribution of the given grid rows to y (or gs), so a caller may
 * feed the grid in row chunks.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* v[g][b][n] for the rows of the chunk: eq. (1) then D_t */
static void seafloor_velocity(int64_t nrows, int64_t nsub, int64_t nt, double dt, int diff,
                              const double* G, int64_t B, const double* s, double* v) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t g = 0; g < nrows; g++) {
    double* m = (double*)malloc(sizeof(double) * (size_t)nt);
    for (int64_t b = 0; b < B; b++) {
      /* eq. (1): m_g[n] = sum_j sum_{k=0}^{n} G[g][j][k] s[b][j][n-k] */
      for (int64_t n = 0; n < nt; n++) m[n] = 0.0;
      for (int64_t j = 0; j < nsub; j++) {
        const double* gk = G + (g * nsub + j) * nt;
        const double* sj = s + (b * nsub + j) * nt;
        for (int64_t k = 0; k < nt; k++) {
          const double gv = gk[k];
          for (int64_t n = k; n < nt; n++) m[n] += gv * sj[n - k];
        }
      }
      /* D_t */
      double* vg = v + (g * B + b) * nt;
      for (int64_t n = 0; n < nt; n++) {
        if (diff) vg[n] = (m[n] - (n > 0 ? m[n - 1] : 0.0)) / dt;
        else vg[n] = m[n];
      }
    }
    free(m);
  }
}

void s2w_oracle_forward_accum(int64_t nrows, int64_t nsub, int64_t nobs, int64_t nt, double dt, int32_t diff,
                              const double* G, const double* F, int64_t B, const double* s, double* y) {
  if (nrows <= 0 || B <= 0) return;
  double* v = (double*)malloc(sizeof(double) * (size_t)(nrows * B * nt));
  seafloor_velocity(nrows, nsub, nt, dt, diff, G, B, s, v);
  /* eq. (2): y[b][o][n] += sum_g sum_{k=0}^{n} F[g][o][k] v[g][b][n-k] */
#pragma omp parallel for collapse(2) schedule(static)
  for (int64_t b = 0; b < B; b++) {
    for (int64_t o = 0; o < nobs; o++) {
      double* yo = y + (b * nobs + o) * nt;
      for (int64_t g = 0; g < nrows; g++) {
        const double* fk = F + (g * nobs + o) * nt;
        const double* vg = v + (g * B + b) * nt;
        for (int64_t k = 0; k < nt; k++) {
          const double fv = fk[k];
          for (int64_t n = k; n < nt; n++) yo[n] += fv * vg[n - k];
        }
      }
    }
  }
  free(v);
}

void s2w_oracle_adjoint_accum(int64_t nrows, int64_t nsub, int64_t nobs, int64_t nt, double dt, int32_t diff,
                              const double* G, const double* F, int64_t B, const double* r, double* gs) {
  if (nrows <= 0 || B <= 0) return;
  double* wp = (double*)malloc(sizeof(double) * (size_t)(nrows * B * nt));
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t g = 0; g < nrows; g++) {
    double* w = (double*)malloc(sizeof(double) * (size_t)nt);
    for (int64_t b = 0; b < B; b++) {
      /* transpose of eq. (2): w[n] = sum_o sum_{k=0}^{nt-1-n} F[g][o][k] r[b][o][n+k] */
      for (int64_t n = 0; n < nt; n++) w[n] = 0.0;
      for (int64_t o = 0; o < nobs; o++) {
        const double* fk = F + (g * nobs + o) * nt;
        const double* ro = r + (b * nobs + o) * nt;
        for (int64_t k = 0; k < nt; k++) {
          const double fv = fk[k];
          for (int64_t n = 0; n + k < nt; n++) w[n] += fv * ro[n + k];
        }
      }
      /* D_t transposed */
      double* wg = wp + (g * B + b) * nt;
      for (int64_t n = 0; n < nt; n++) {
        if (diff) wg[n] = (w[n] - (n + 1 < nt ? w[n + 1] : 0.0)) / dt;
        else wg[n] = w[n];
      }
    }
    free(w);
  }
  /* transpose of eq. (1): gs[b][j][n] += sum_g sum_{k=0}^{nt-1-n} G[g][j][k] w'[g][b][n+k] */
#pragma omp parallel for collapse(2) schedule(static)
  for (int64_t b = 0; b < B; b++) {
    for (int64_t j = 0; j < nsub; j++) {
      double* gj = gs + (b * nsub + j) * nt;
      for (int64_t g = 0; g < nrows; g++) {
        const double* gk = G + (g * nsub + j) * nt;
        const double* wg = wp + (g * B + b) * nt;
        for (int64_t k = 0; k < nt; k++) {
          const double gv = gk[k];
          for (int64_t n = 0; n + k < nt; n++) gj[n] += gv * wg[n + k];
        }
      }
    }
  }
  free(wp);
}

/*
 * One block lower-triangular Toeplitz matvec in the form of eq. (4):
 * y[b][i][n] = sum_j sum_{k=0}^{n} K[i][j][k] x[b][j][n-k]   (trans = 0)
 * and its transpose
 * x[b][j][n] = sum_i sum_{k=0}^{nt-1-n} K[i][j][k] y[b][i][n+k]   (trans = 1).
 * K[i][j][k] = [F_k]_{i,j}.  Overwrites the output.
 */
void s2w_oracle_bltt(int64_t nout, int64_t nin, int64_t nt, const double* K, int64_t B, int32_t trans,
                     const double* in, double* out) {
  if (!trans) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t b = 0; b < B; b++)
      for (int64_t i = 0; i < nout; i++) {
        double* yi = out + (b * nout + i) * nt;
        for (int64_t n = 0; n < nt; n++) yi[n] = 0.0;
        for (int64_t j = 0; j < nin; j++) {
          const double* kk = K + (i * nin + j) * nt;
          const double* xj = in + (b * nin + j) * nt;
          for (int64_t n = 0; n < nt; n++) {
            double acc = 0.0;
            for (int64_t k = 0; k <= n; k++) acc += kk[k] * xj[n - k];
            yi[n] += acc;
          }
        }
      }
  } else {
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t b = 0; b < B; b++)
      for (int64_t j = 0; j < nin; j++) {
        double* xj = out + (b * nin + j) * nt;
        for (int64_t n = 0; n < nt; n++) xj[n] = 0.0;
        for (int64_t i = 0; i < nout; i++) {
          const double* kk = K + (i * nin + j) * nt;
          const double* yi = in + (b * nout + i) * nt;
          for (int64_t n = 0; n < nt; n++) {
            double acc = 0.0;
            for (int64_t k = 0; k + n < nt; k++) acc += kk[k] * yi[n + k];
            xj[n] += acc;
          }
        }
      }
  }
}
