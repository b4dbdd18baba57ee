// Exact sparse solver for the Schur complement of the constraint
// preconditioner: LU factorisation without pivoting, built on the host in
// FP64 (multifrontal, nested-dissection order), applied on the device level
// by level of the dissection tree.
#pragma once

#include "common.h"

namespace sie {

struct SparseLU {
    int64_t n = 0;                     // unknowns
    int nsn = 0;                       // supernodes (leaves and separators)
    int max_sn = 0;                    // largest supernode
    std::vector<int> lev_ptr;          // supernodes of level l: lev_sn[lev_ptr[l] .. lev_ptr[l + 1])
    DBuf<int32_t> lev_sn;              // supernode ids grouped by level (leaves first)
    DBuf<int32_t> sn_p0, sn_n;         // first position and size of each supernode
    DBuf<int64_t> inv_off;             // offset of a supernode's n x n inverse blocks
    DBuf<c128> linv, uinv;             // inverses of its unit-lower and upper diagonal blocks
    DBuf<int64_t> lrow_ptr, urow_ptr;  // off-block entries per position (row) of L and U
    DBuf<int32_t> lcol, ucol;
    DBuf<c128> lval, uval;
    DBuf<int32_t> perm, iperm;         // position -> unknown, unknown -> position
    int64_t nnz_factor = 0;            // stored off-block entries of L and U
    double t_factor_s = 0.0;
    double est_flops = 0.0;            // arithmetic of the factorisation
    // row blocks of the device solve: block b of level l (blk_ptr[l] <= b <
    // blk_ptr[l + 1]) takes rows blk_row0[b] .. + kLURowsPerBlock - 1 of
    // supernode blk_sn[b]
    std::vector<int> blk_ptr;
    DBuf<int32_t> blk_sn, blk_row0;
    mutable DBuf<c128> work;           // [nrhs][n] gathered right-hand sides of a level
    // FP32 copies of the factors for FP32 solves (lu_make_fp32)
    DBuf<c64> linv32, uinv32, lval32, uval32;
    mutable DBuf<c64> work32;
};
// Rows of one supernode per workgroup of the device solve (one wavefront each).
constexpr int kLURowsPerBlock = 4;

// Factor the n x n matrix in CSR (rp, ci sorted per row, val); its pattern
// must be structurally symmetric.  coords [n][3] place the unknowns in space
// for the dissection.  The ordering and the symbolic factorisation run on
// the host, the numeric one on the device (stream st, synchronised before
// returning) or, with small fronts only, on the host.  Throws SIE_EINVAL when a separator exceeds kLUMaxSupernode
// unknowns, when the factors would exceed kLUMaxBytes of device memory or
// kLUMaxFlops of arithmetic (estimated before any front is factored), or
// when a pivot vanishes.
constexpr int kLUMaxSupernode = 4096;
constexpr double kLUMaxBytes = 8e9;
constexpr double kLUMaxFlops = 5e12;
// Factorisations whose fronts all have at most kLUHostFront rows run on the
// host (launches would dominate their device time).
constexpr int kLUHostFront = 512;
void lu_factor(SparseLU &f, int64_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &ci,
               const std::vector<c128> &val, const std::vector<double> &coords, hipStream_t st);

// Rounds the factors to FP32 copies (for lu_solve on complex64 vectors).
void lu_make_fp32(SparseLU &f, hipStream_t st);

// x [nrhs][n] in position order: overwritten by the solution of (LU) x = b,
// in FP64, or in FP32 with the FP32 copies of the factors.
void lu_solve(const SparseLU &f, int nrhs, c128 *x, hipStream_t st);
void lu_solve(const SparseLU &f, int nrhs, c64 *x, hipStream_t st);

// xp[r][iperm[j]] = x[r * E + r0 + j], j < n: rows [r0, r0 + n) of nrhs
// vectors into position order.
template <typename T>
void launch_lu_gather(int64_t n, int64_t r0, int64_t E, int nrhs, const int32_t *iperm, const cx<T> *x, cx<T> *xp,
                      hipStream_t st);
// y[r * E + r0 + j] = xp[r][iperm[j]].
template <typename T>
void launch_lu_scatter(int64_t n, int64_t r0, int64_t E, int nrhs, const int32_t *iperm, const cx<T> *xp, cx<T> *y,
                       hipStream_t st);

// One front of the numeric factorisation (k_front.hip), in stream order:
// F [m][m] (row-major, device) is cleared, receives its original entries
// (F[arow[e]][acol[e]] = val[asrc[e]], e < nasm) and adds each child's update
// matrix (child_upd [bc][bc], its rows and columns at child_map [bc] of F);
// its first n positions are then eliminated without pivoting, linv and uinv
// [n][n] receive the inverses of the unit-lower L_NN and the upper U_NN,
// row a of L_BN goes to lval[loff[a] ..] and row k of U_NB to
// uval[urow[k] ..], and the Schur complement on the boundary to upd
// [nb][nb] (nb = m - n; none when nb = 0).  *bad is set non-zero on a pivot
// that is zero or not finite.
struct FrontStep {
    c128 *F = nullptr;
    int m = 0, n = 0;
    const int32_t *arow = nullptr, *acol = nullptr, *asrc = nullptr;
    int64_t nasm = 0;
    const c128 *val = nullptr;
    std::vector<const c128 *> child_upd;
    std::vector<int> child_nb;
    std::vector<const int32_t *> child_map;
    c128 *linv = nullptr, *uinv = nullptr;
    c128 *lval = nullptr;
    const int64_t *loff = nullptr;
    c128 *uval = nullptr;
    const int64_t *urow = nullptr;
    c128 *upd = nullptr;
    int *bad = nullptr;
};
void launch_front_step(const FrontStep &s, hipStream_t st);

// Device side (k_lu.hip): one level of the forward or backward sweep, two
// launches (gather the solved levels' contributions into f.work, then the
// dense inverses of the diagonal blocks), rows spread over workgroups.
// T = float uses the FP32 copies of the factors.
template <typename T>
void launch_lu_level(const SparseLU &f, int level, bool forward, int nrhs, cx<T> *x, hipStream_t st);

}  // namespace sie
