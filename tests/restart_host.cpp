// Host harness for the long-cycle Krylov dense steps (the restart, the column update and the
// least-squares solve of bigkrylov.h), run on one host thread.  Used by
// tests/test_restart_host.py, which compares the results with the oracle.
//
//   restart_host restart IN OUT   IN: int m, k, final; Hbar (m+1) x m, c (m+1), u (m+1) (complex
//                                 doubles, column-major); OUT: int status, nrot; double est;
//                                 kept eigenvalues (k); P (m+1) x (k+1); Hbar_k (k+1) x k;
//                                 c (k+1); g (k+1)
//   restart_host columns IN OUT   IN: int m, k; Hbar (m+1) x m; beta; then int m2 and the
//                                 columns k .. m2-1 of a second Hessenberg matrix appended after a
//                                 restart of the first (m2 + 1 rows each); OUT: per phase int
//                                 steps; double est; y (steps)
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../paper_1912_02868_amd/csrc/bigkrylov.h"

using namespace dmg;

static void rd(FILE* f, void* p, size_t n) {
  if (fread(p, 1, n, f) != n) {
    fprintf(stderr, "short read\n");
    exit(2);
  }
}

int main(int argc, char** argv) {
  if (argc != 4) return 2;
  FILE* in = fopen(argv[2], "rb");
  FILE* out = fopen(argv[3], "wb");
  if (!in || !out) return 2;
  KBig* kb = (KBig*)calloc(1, sizeof(KBig));
  std::vector<double2> work(big_restart_work_elems());
  std::vector<double2> shm(2 * LDBIG + 16);
  HostTeam tm{shm.data()};
  int hdr[3];
  if (!strcmp(argv[1], "restart")) {
    rd(in, hdr, sizeof(hdr));
    const int m = hdr[0], k = hdr[1], fin = hdr[2];
    for (int j = 0; j < m; ++j) rd(in, kb->H + LDBIG * j, sizeof(double2) * (m + 1));
    rd(in, kb->c, sizeof(double2) * (m + 1));
    rd(in, kb->u, sizeof(double2) * (m + 1));
    std::vector<double2> P((size_t)(m + 1) * (k + 1));
    const int st = big_restart_body(tm, kb, m, k, P.data(), fin, work.data());
    const double2* lam = work.data() + 6 * LDBIG * LDBIG + LDBIG;
    const int* order = (const int*)(lam + LDBIG);
    fwrite(&st, sizeof(int), 1, out);
    fwrite(&kb->nrot, sizeof(int), 1, out);
    fwrite(&kb->est, sizeof(double), 1, out);
    for (int q = 0; q < k; ++q) fwrite(&lam[order[q]], sizeof(double2), 1, out);
    fwrite(P.data(), sizeof(double2), P.size(), out);
    for (int j = 0; j < k; ++j) fwrite(kb->H + LDBIG * j, sizeof(double2), k + 1, out);
    fwrite(kb->c, sizeof(double2), k + 1, out);
    fwrite(kb->g, sizeof(double2), k + 1, out);
  } else if (!strcmp(argv[1], "columns")) {
    rd(in, hdr, 2 * sizeof(int));
    const int m = hdr[0], k = hdr[1];
    std::vector<double2> Hb((size_t)(m + 1) * m);
    rd(in, Hb.data(), sizeof(double2) * Hb.size());
    double beta;
    rd(in, &beta, sizeof(double));
    // a fresh cycle: c = g = beta e1
    kb->c[0] = kb->g[0] = mk(beta, 0.0);
    kb->tol_abs = 0.0;
    for (int j = 0; j < m; ++j) {
      for (int i = 0; i <= j; ++i) {
        kb->h1[i] = Hb[i + (m + 1) * j];
        kb->h2[i] = mk(0.0, 0.0);
      }
      kb->wn = cabs2(Hb[j + 1 + (m + 1) * j]);
      kb->wn0 = 1.0;
      big_column_body(tm, kb, j);
    }
    big_lssolve_body(tm, kb);
    fwrite(&kb->steps, sizeof(int), 1, out);
    fwrite(&kb->est, sizeof(double), 1, out);
    fwrite(kb->y, sizeof(double2), kb->steps, out);
    // restart to k vectors, then append the columns k .. m2-1 of a second matrix
    std::vector<double2> P((size_t)(m + 1) * (k + 1));
    const int st = big_restart_body(tm, kb, m, k, P.data(), 0, work.data());
    int m2;
    rd(in, &m2, sizeof(int));
    std::vector<double2> H2((size_t)(m2 + 1) * m2);
    rd(in, H2.data(), sizeof(double2) * H2.size());
    for (int j = k; j < m2; ++j) {
      for (int i = 0; i <= j; ++i) {
        kb->h1[i] = H2[i + (m2 + 1) * j];
        kb->h2[i] = mk(0.0, 0.0);
      }
      kb->wn = cabs2(H2[j + 1 + (m2 + 1) * j]);
      kb->wn0 = 1.0;
      big_column_body(tm, kb, j);
    }
    big_lssolve_body(tm, kb);
    fwrite(&st, sizeof(int), 1, out);
    fwrite(P.data(), sizeof(double2), P.size(), out);
    for (int j = 0; j < k; ++j) fwrite(kb->H + LDBIG * j, sizeof(double2), k + 1, out);
    fwrite(kb->c, sizeof(double2), k + 1, out);
    fwrite(&kb->steps, sizeof(int), 1, out);
    fwrite(&kb->est, sizeof(double), 1, out);
    fwrite(kb->y, sizeof(double2), kb->steps, out);
  } else {
    return 2;
  }
  fclose(out);
  fclose(in);
  free(kb);
  return 0;
}
