// Launchers of the solve kernels (k_solve.hip).
#pragma once
#include "problem.h"

namespace sie {
void launch_excitation(sie_problem *p, const double *rule, int nq, double k0, const double khat[3], const c128 e0[3],
                       c128 *out, hipStream_t st);
void launch_farfield(sie_problem *p, const double *rule, int nq, double k0, double eta0, const double *rhat,
                     int64_t ndir, const c128 *u, const c128 *v, c128 *F, hipStream_t st);
void launch_bj_setup(int nb, int B, const int32_t *perm, int64_t rwg0, const int64_t *row_ptr, const int32_t *cols,
                     const c128 *vals, c128 scale, c128 *inv64, c64 *inv32, hipStream_t st);
template <typename T>
void launch_bj_apply(int nb, int B, const int32_t *perm, const cx<T> *inv, const cx<T> *x, cx<T> *y, hipStream_t st);
// Schwarz clusters of the near-region preconditioner: largest extended
// cluster (RWG functions) the kernels take.
constexpr int kRasMax = 2048;
// Near-field rows of one medium that its clusters' matrices come from:
// scale * vals of the CSR rows (RWG rwg0 + r).
struct RasSource {
    int64_t rwg0;
    const int64_t *row_ptr;
    const int32_t *cols;
    const c128 *vals;
    c128 scale;
};
// Clusters c0 .. c0 + cnt - 1 (cluster c's rows from src[cmed[c]]); their
// workspaces start at ws + ws_off[c] - ws_off[c0].
void launch_ras_setup(int c0, int cnt, const int64_t *ext_off, const int32_t *ext, const int32_t *own_off,
                      const int32_t *own_pos, const int64_t *ws_off, const int64_t *m_off, const int32_t *cmed,
                      const RasSource *src, c128 *ws, c128 *m64, c64 *m32, int *fail, hipStream_t st);
// active (optional, [nrhs][nobj]): clusters whose object cobj[c] is
// inactive for a right-hand side write zeros to their owned rows.
template <typename T>
void launch_ras_apply(int nc, int max_own, const int64_t *ext_off, const int32_t *ext, const int32_t *own_off,
                      const int32_t *own, const int64_t *m_off, const cx<T> *M, const cx<T> *x, cx<T> *y, int64_t ld,
                      int nrhs, hipStream_t st, const uint8_t *active = nullptr, int nobj = 0,
                      const int32_t *cobj = nullptr);
}  // namespace sie
