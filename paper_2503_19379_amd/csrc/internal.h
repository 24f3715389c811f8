// Internal launch interfaces of the mfdkc HIP library.
#pragma once
#include <hip/hip_runtime.h>

namespace mfd {

// Per-call operator parameters: grid, Bloch vector, penalty and shift.
struct OpParams {
    int N;
    double L, h;
    double k[3];
    double gamma, shift;
    int order = 2;             // stencil order 2K (Table FD_1D)
    int stencil_wgs = 2048;    // order 2: z chunks until this many workgroups (N = 64: waves)
    int fft_xc = 0;            // x run of the z-pass of the FFT solve (0: the largest of 16, 8, 4, 2, 1 dividing N)
    void* wtmp = nullptr;      // two-pass operator: scratch for wtmp_bands bands of 4 FP64 complex fields
    int wtmp_bands = 0;
    // General lattice (Section 4.2, eq. (coordinate_change)): the grid is the
    // unit cube of y = A^-1 x and D^_i = sum_j b_ji K_j + i L_i.  B[i][j] =
    // N b_ji weighs the unit-step difference along grid axis j in D^_i.
    int lattice = 0;
    double B[3][3] = {};
};

// Weight of the unit-step difference along grid axis j in D_i: B[i][j] on a
// general lattice, 1/h on the diagonal of a cubic one.
inline double diff_weight(const OpParams& p, int i, int j) {
    return p.lattice ? p.B[i][j] : (i == j ? 1.0 / p.h : 0.0);
}

// Orders > 2 and general lattices use the two-pass operator.
inline bool two_pass(const OpParams& p) { return p.order > 2 || p.lattice; }

// Table FD_1D coefficients (c_s, d_s), s = 1..order/2, zero-padded to 4 (wide.hip).
void stencil_coefs(int order, double c[4], double d[4]);

// Which fields of a block a launch processes: field b of the launch is field
// idx[b] of the block when a list is given (at most 32), else field b.
struct FieldList {
    unsigned char idx[32];
    int on = 0;
    __host__ __device__ int operator()(int b) const { return on ? idx[b] : b; }
};

// Y = (A M_0 A' + gamma B'B + shift I) X for nb fields (stencil.hip).
template <class R>
hipError_t launch_stencil(const OpParams& p, int nb, const void* X, void* Y, const void* mu, hipStream_t s,
                          const FieldList& fl = FieldList());

// Orders > 2 and general lattices: the same operator in two passes through
// p.wtmp (wide.hip); R arithmetic, S storage.
template <class R, class S>
hipError_t launch_wide(const OpParams& p, int nb, const void* X, void* Y, const void* mu, hipStream_t s,
                       const FieldList& fl);

// General lattice, order 2: the same operator in one z-marching pass with
// v, e and q tiles in LDS (lattice.hip); launch_wide calls it.
template <class R, class S>
hipError_t launch_lattice(const OpParams& p, int nb, const void* X, void* Y, const void* mu, hipStream_t s,
                          const FieldList& fl);

// Same operator with FP64 arithmetic on FP32-stored fields (c64 in, c64 out).
hipError_t launch_stencil_f64_s32(const OpParams& p, int nb, const void* X, void* Y, const void* mu64,
                                  hipStream_t s, const FieldList& fl = FieldList());

// T = (P + shift I)^-1 R for nb fields via FFT (fft.hip).  tw: device table
// exp(-2 pi i j / N), j < N, of precision R.
template <class R>
hipError_t launch_precond(const OpParams& p, int nb, const void* Rin, void* Tout, const void* tw, hipStream_t s,
                          const FieldList& fl = FieldList());
bool fft_supported(int N, int real_bytes);
// the x-y plane pass holds a whole plane in LDS (else it runs as separate x
// and y passes, two more reads and writes of the block)
bool fft_plane_fits(int N, int real_bytes);
// FP32 register-resident passes (fft_reg.hip): cubic order-2 contexts of N = 16, 32, 64
bool reg_precond_ok(const OpParams& p);
hipError_t launch_precond_reg(const OpParams& p, int nb, const void* Rin, void* Tout, const void* tw, hipStream_t s,
                              const FieldList& fl = FieldList());

// Multigrid solve of the same system (mg.hip; Section 5.3, Alg 5.2): cubic
// order-2 contexts whose grid halves down to at most 5^3 cells.
struct MGOpts {
    int cycles = 2;   // V-cycles per scalar solve, from a zero guess
    int n1 = 2, n2 = 2;   // pre- and post-smoothing steps
    int sweeps = 2;   // Jacobi sweeps per triangular factor in a smoothing step
};
struct MGWork;
MGWork* mg_create();
void mg_destroy(MGWork* w);
bool mg_supported(int N);
template <class S>
hipError_t launch_precond_mg(MGWork* w, const OpParams& p, const MGOpts& o, int nb, const void* Rin, void* Tout,
                             hipStream_t s, const FieldList& fl = FieldList());

// out[b] = sum mu |A' x_b|^2 and out[nb + b] = sum |x_b|^2, c128 fields (blas.hip).
hipError_t launch_lambda_re(const OpParams& p, int nb, const void* X, const void* mu, double* partial,
                            int nparts, double* out, hipStream_t s);

}  // namespace mfd
