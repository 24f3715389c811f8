// Learned warm start of the band solve along a k-path: the network (mlp.hip)
// and the per-workspace state that builds its training pairs and proposals
// (warm.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/mfdkc.h"

namespace mfd {

struct Mlp {
    int nin = 0, nh = 0, nl = 0, nout = 0, bmax = 0;
    bool bf16 = true;          // products read the bfloat16 copy (else the FP32 master)
    int t = 0;                 // Adam steps taken
    size_t nparam = 0;
    std::vector<int> dims;     // nin, nh x nl, nout
    std::vector<size_t> woff;  // offset of each layer's W in the flat vector (b follows W)
    float* p = nullptr;        // FP32 master parameters
    float* g = nullptr;        // gradient of the last loss_grad
    float* m = nullptr;        // Adam moments
    float* v = nullptr;
    void* pb = nullptr;        // bfloat16 copy of p
    float* work = nullptr;     // activations and backward buffers for bmax rows
    double* dloss = nullptr;   // loss of the last loss_grad (device)

    int init(int nin, int nh, int nl, int nout, int bmax, bool bf16, uint64_t seed);
    int set_params(const float* host, hipStream_t s);
    int randomize(uint64_t seed, hipStream_t s);   // the initial parameters; clears Adam
    void release();
    float* act_in(int l) const;
    float* pre(int l) const;
    float* grad_buf(int which) const;
    hipError_t forward(int B, const float* X, float* Y, hipStream_t s);
    hipError_t loss_grad(int B, const float* X, const float* T, hipStream_t s);
    hipError_t adam(float lr, hipStream_t s);
};

// Warm start from the blocks of the previous k-points (one per workspace).
// Roles: a = X_{j-1}, b = X_j, c = X_{j+1}, the three latest converged blocks.
struct WarmStart {
    int mb = 0;
    size_t n = 0;
    double L = 1.0;              // cell side (feature scaling)
    int nin = 0, nout = 0, pmax = 64;
    double2* H = nullptr;        // n x 3mb: three history slots of mb columns, each stored
                                 // aligned (Procrustes) with the block before it
    double2* G = nullptr;        // 3mb x 3mb Gram of the slots
    double2* gpart = nullptr;
    int nparts = 0;
    double2* Cb = nullptr;       // C* of the latest pair (2mb x mb)
    double2* Cc = nullptr;       // C* being formed
    double2* Rinv = nullptr;     // R^-1 of orth[X_c Q, X_b] (2mb x 2mb), for the next proposal
    double2* Qc = nullptr;       // polar factor aligning X_c with X_b (mb x mb)
    double2* D = nullptr;        // proposal coefficients (2mb x mb)
    float* F = nullptr;          // replay buffer: features (pmax x nin)
    float* T = nullptr;          //                targets  (pmax x nout)
    float* feat = nullptr;       // one feature row
    float* pred = nullptr;       // one network output row
    int* dstatus = nullptr;
    float* hstage = nullptr;     // pinned: feature head
    int* hstatus = nullptr;      // pinned
    int slot[3] = {0, 1, 2};     // role -> history slot
    double lam[3][32];           // Ritz values per slot
    double kk[3][3];             // k per slot
    int nsolved = 0, npairs = 0, pnext = 0;
    uint64_t seed = 0;
    bool have_cb = false;        // Cb holds C* of the pair ending at X_b
    bool rinv_ok = false;
    // held-out error ratios (network / no change) of the latest pairs, each
    // measured before the network trained on that pair
    double score[4] = {0, 0, 0, 0};
    int nscore = 0;
    bool last_used_net = false;  // the last proposal applied the network's correction
    float* zeros = nullptr;      // a zero output row
    double* dsq = nullptr;
    double* hsq = nullptr;       // pinned
    Mlp net;

    int init(size_t n, int mb, double L, uint64_t seed);
    void release();
    int reset(hipStream_t s);   // empty history and replay buffer, initial network
    // After a solve at k with converged block X (n x mb c128, column-major) and Ritz values.
    int after_solve(const double2* X, const double* theta, const double* k, int steps, float lr, hipStream_t s);
    // Writes the proposed start block for k_next into W (c128, or c64 when w32); false if not ready.
    int propose(const double* k_next, void* W, bool w32, bool* made, hipStream_t s);
    // the network's correction is applied while its recent held-out error is
    // below 0.8 of the no-change error
    bool net_trusted() const;
};

hipError_t launch_warm_target(const double2* G, int mb, int a, int b, int c, double2* Cout, double2* Qout,
                              double2* Rinv, int* status, hipStream_t s);
hipError_t warm_feature_row(double L, int mb, const double* k_prev, const double* k_next, const double* lam_j,
                            const double* lam_jm1, const double2* Cj, float* row, float* stage, hipStream_t s);
int warm_target_blocks(size_t n, int mb, const double2* Xa, const double2* Xb, const double2* Xc, double2* C,
                       double2* Rinv, hipStream_t s);

}  // namespace mfd
