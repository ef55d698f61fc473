/* tlfea_oracle_omp.c -- timing-only OpenMP form of the oracle's fused f + K.
 *
 * TEST INFRASTRUCTURE ONLY (the benchmark's CPU-baseline leg times it on all
 * host cores).  It compiles the single-threaded oracle unchanged and adds one
 * entry point that runs the same element loop (Sec. 4.3, Eqs. fint_local /
 * atomic_scatter; Sec. 4.4.2, Eq. tangent_block) over threads, scattering with
 * atomic adds as the paper's kernels do.  Correctness is the single-threaded
 * oracle's; this form only gives a multi-core time.
 */
#include "tlfea_oracle.c"

#include <omp.h>

int orc_omp_threads(void) { return omp_get_max_threads(); }

int orc_assemble_omp(const orc_mesh* mesh, const orc_material* mat, const double* q, const double* qdot,
                     double alpha, double beta, double* f, const int* row_off, const int* cols, double* vals) {
  const int nen = orc_n_en(mesh->elem_type);
  const int nd = 3 * nen;
  const mat_int mi = to_internal(mat);
  int rc = ORC_OK;
#pragma omp parallel
  {
    double* fe = (double*)malloc(sizeof(double) * nd);
    double* Ke = (double*)malloc(sizeof(double) * nd * nd);
    int my_rc = ORC_OK;
#pragma omp for schedule(static)
    for (int e = 0; e < mesh->n_elem; ++e) {
      if (my_rc != ORC_OK) continue;
      memset(fe, 0, sizeof(double) * nd);
      memset(Ke, 0, sizeof(double) * nd * nd);
      my_rc = element_int(mesh, &mi, e, q, qdot, alpha, beta, fe, Ke);
      if (my_rc != ORC_OK) continue;
      for (int a = 0; a < nen; ++a) {
        const int ca = coef_of(mesh, e, a);
        for (int i = 0; i < 3; ++i) {
#pragma omp atomic
          f[3 * ca + i] += fe[3 * a + i];
          for (int b = 0; b < nen; ++b) {
            const int cb = coef_of(mesh, e, b);
            for (int kk = 0; kk < 3; ++kk) {
              const long long pos = find_col(row_off, cols, 3 * ca + i, 3 * cb + kk);
              if (pos < 0) { my_rc = ORC_ENOTFOUND; break; }
#pragma omp atomic
              vals[pos] += Ke[(3 * a + i) * nd + 3 * b + kk];
            }
          }
        }
      }
    }
    free(fe);
    free(Ke);
#pragma omp critical
    if (my_rc != ORC_OK) rc = my_rc;
  }
  return rc;
}
