// Internal launchers of the block eigensolver (blas.hip, rr.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdint>

namespace mfd {

hipError_t launch_reduce(const double* parts, int nparts, int ncols, double* out, hipStream_t s);
// G (P x Q, row-major c128) = V[:, :P]^H V[:, :Q], V column-major with leading dimension ld.
hipError_t launch_gram(const void* V, size_t ld, size_t n, int P, int Q, int nparts, void* part, void* G,
                       hipStream_t s);
int gram_parts(size_t n);
hipError_t launch_update(const void* V, void* U, size_t ld, size_t n, int mb, const void* C, const double* theta,
                         int nparts, double* npart, double* norms, hipStream_t s);
// The basis of one Rayleigh-Ritz step: X (mb columns), the W columns of the
// na unconverged bands and the np P columns of those bands, K = mb + na + np, with the images AX, AW, AP at basis columns K..2K.  V holds
// [X | W | P | AX | AW | AP], mb columns each, in band order.
constexpr int BASIS_KMAX = 66;   // 3 x the largest block (22 columns)
struct BasisMap {
    int mb, K, na;
    short lc[2 * BASIS_KMAX];  // load ordinal -> basis column (FP64 columns first in mixed precision)
    short pc[2 * BASIS_KMAX];  // load ordinal -> column of V
    signed char tpos[32];      // band -> its W column among the na (-1: converged)
    unsigned char act[32];     // W column t -> band
};

// MFMA (FP64 matrix core) versions: Gram of the K basis columns against
// [S | AS] (Hermitian halves only), and the block update (gemm.hip).
// V32 (or null): FP32 storage of the W, P, AW, AP columns (mixed precision).
// stages: 1 the tile kernel (per-workgroup partial tiles), 2 their fixed-order
// sum and the Hermitian scatter into G, 3 both.
hipError_t launch_gram_mfma(const void* V, const void* V32, size_t ld, size_t n, const BasisMap& bm, int nparts,
                            void* part, void* G, hipStream_t s, int stages = 3);
int gram_mfma_parts(size_t n);
size_t gram_mfma_part_elems(int K, int nparts);
// U = [X' | R' | P' | AX' | - | AP'] from the K x mb coefficients C, every
// band.  U32 (or null): FP32 outputs R', P', AP' (mixed precision).
// rows: 0 one wave per 16-row strip; 16 or 32 rows per workgroup block.
hipError_t launch_update_mfma(const void* V, const void* V32, void* U, void* U32, size_t ld, size_t n,
                              const BasisMap& bm, const void* C, const double* theta, int nparts, double* npart,
                              double* norms, hipStream_t s, int rows = 0, bool sum = true);
// R = AX - X theta written to W (FP32 if R32), column norms |R|^2, |X|^2 (blas.hip).
hipError_t launch_residual(const void* X, const void* AX, void* R, bool r32, size_t ld, size_t n, int mb,
                           const double* theta, int nparts, double* npart, double* norms, hipStream_t s);
hipError_t launch_colstats(const void* X, const void* Y, size_t ld, size_t n, int nb, const double* theta,
                           int nparts, double* part, double* out, hipStream_t s);
hipError_t launch_fill_random(void* X, size_t count, uint64_t seed, hipStream_t s);
// Cold start from plane waves: column j of X (n = 3 N^3 rows, c128) becomes
// pol[j] exp(2 pi i m_j . r / N) plus `noise` times the column's present
// (random) values.
struct PlaneWaves {
    int mb;
    int m[22][3];
    double2 pol[22][3];
};
hipError_t launch_planewave_start(void* X, int N, const PlaneWaves& pw, double noise, hipStream_t s);
hipError_t launch_convert(const void* X, void* Y, size_t count, bool to_c64, hipStream_t s);

// Rayleigh-Ritz on span[X, W, P] (rr.hip) for a basis of K = mb + nw + np
// columns: X (mb), then the nw W columns and the np P columns of the
// unconverged bands.
//   G:      K x 2K row-major c128, [S^H S | S^H A S]
//   theta:  mb doubles, the new Ritz values (out)
//   C:      K x mb row-major c128 coefficients (out)
//   info:   ints (out): [0] = columns kept, [1] = 1 if a P column was dropped,
//           [2] = active bands (nw), [3] = Jacobi sweeps, [4..8] phase ticks, [9] = kept
struct RRArgs {
    const double2* G;
    double* theta;
    double2* C;
    int* info;
    double* floor;   // (out) Kv eps max|eig(H)|: the absolute accuracy of a Householder-route Ritz value
    int mb, K, nw;
    double drop_w, drop_p;
};
hipError_t launch_rr(const RRArgs& a, hipStream_t s);
// The same step with cyclic Jacobi on H (rr_jacobi.hip): slower, and accurate
// relative to the Ritz values themselves; the solver takes it in its last
// iterations, where rr.hip's absolute accuracy would bound the residual.
hipError_t launch_rr_jacobi(const RRArgs& a, hipStream_t s);

// Hard locking of the last iterations (lock.hip).  LK_NA: most bands still
// iterating when it applies; LK_MAXL: most locked bands.
constexpr int LK_NA = 8, LK_MAXK = 3 * LK_NA, LK_MAXL = 22, LK_MAXT = LK_NA;
// Columns of c = X_L^H Y and of Y -= X_L c (Z -= AX_L c with zpair):
// xc / axc: V columns of X_L and AX_L; yc / zc: columns of Y and Z (V32 with
// y32, else V).
struct LockCols {
    int nl = 0, nt = 0, y32 = 0, zpair = 0;
    short xc[LK_MAXL], axc[LK_MAXL], yc[LK_MAXT], zc[LK_MAXT];
};
// part: room for nparts + nparts / 64 + 1 sets of nl x nt partial sums
hipError_t launch_lock_coef(const LockCols& c, const void* V, const void* V32, size_t ld, size_t n, int nparts,
                            void* part, void* coef, hipStream_t s);
hipError_t launch_lock_apply(const LockCols& c, const void* coef, void* V, void* V32, size_t ld, size_t n,
                             int nblocks, hipStream_t s);
// Basis [X_A W_A P] of the bands act[0..na) for the hard-locked update: sc /
// ic the columns of basis column k and of its image (V32 when bit k of f32 is
// set, else V); C is K x na (row-major), theta the na Ritz values.
struct LockBasis {
    int na = 0, K = 0, mb = 0;
    unsigned long long f32 = 0;
    short sc[LK_MAXK], ic[LK_MAXK];
    unsigned char act[LK_NA];
};
hipError_t launch_lock_update(const LockBasis& b, const void* V, const void* V32, void* U, void* U32, size_t ld,
                              size_t n, const void* C, const double* theta, int nblocks, double* npart, double* norms,
                              hipStream_t s);

}  // namespace mfd
