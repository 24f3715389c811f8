// Multilayer perceptron of the learned warm start: forward, backward and Adam
// on the device.
//
// x -> gelu(W1 x + b1) -> ... -> gelu(W_L h + b_L) -> W_out h + b_out, with
// gelu(z) = z Phi(z), Phi the normal CDF (exact erf form); loss = mean squared
// error over batch and outputs; Adam (Kingma and Ba) with bias correction.
// Parameters are one flat FP32 master vector (per layer W (out x in,
// row-major), then b).  The three products of a layer (forward Z = A W^T,
// data gradient dZ W, weight gradient dZ^T A) run on bfloat16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulate): the weights are a bfloat16
// copy of the master (rounded to nearest even after every step), and each
// FP32 activation or gradient operand is split into hi + lo bfloat16 parts,
// so that the products carry about 16 bits of the FP32 operand (the
// hi x lo and lo x hi terms are formed, lo x lo is dropped).  A debug mode
// reads the FP32 master and runs the products as FP32 FMA loops.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "common.h"
#include "mlp.h"
#include "solver.h"

namespace mfd {

typedef unsigned short bf16_t;

__host__ __device__ __forceinline__ float bf16_to_f(bf16_t h) {
    unsigned int u = ((unsigned int)h) << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// round to nearest, ties to even (finite inputs)
__host__ __device__ __forceinline__ bf16_t f_to_bf16(float f) {
    unsigned int u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

constexpr int ML_TB = 16;   // batch rows per tile
constexpr int ML_TO = 64;   // outputs (or inputs) per tile
constexpr int ML_KC = 32;   // reduction chunk

// FP32 debug products.  Z = A W^T + b (A: B x I, W: O x I), Aout = gelu(Z)
// (act) or Z.
__global__ __launch_bounds__(256) void linear_fwd_kernel(const float* __restrict__ A, int B, int I,
                                                         const float* __restrict__ W, const float* __restrict__ bias,
                                                         int O, int act, float* __restrict__ Z,
                                                         float* __restrict__ Aout) {
    __shared__ float As[ML_TB][ML_KC + 1];
    __shared__ float Ws[ML_TO][ML_KC + 1];
    const int tid = threadIdx.x;
    const int o0 = blockIdx.x * ML_TO, b0 = blockIdx.y * ML_TB;
    const int ol = tid % ML_TO, bg = tid / ML_TO;   // 4 groups of 4 batch rows
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < I; k0 += ML_KC) {
        for (int e = tid; e < ML_TB * ML_KC; e += 256) {
            const int r = e / ML_KC, c = e % ML_KC;
            As[r][c] = (b0 + r < B && k0 + c < I) ? A[(size_t)(b0 + r) * I + k0 + c] : 0.f;
        }
        for (int e = tid; e < ML_TO * ML_KC; e += 256) {
            const int r = e / ML_KC, c = e % ML_KC;
            Ws[r][c] = (o0 + r < O && k0 + c < I) ? W[(size_t)(o0 + r) * I + k0 + c] : 0.f;
        }
        __syncthreads();
#pragma unroll 8
        for (int c = 0; c < ML_KC; ++c) {
            const float w = Ws[ol][c];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = fmaf(As[bg * 4 + q][c], w, acc[q]);
        }
        __syncthreads();
    }
    const int o = o0 + ol;
    if (o >= O) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int b = b0 + bg * 4 + q;
        if (b >= B) continue;
        const float z = acc[q] + bias[o];
        Z[(size_t)b * O + o] = z;
        Aout[(size_t)b * O + o] = act ? gelu_f(z) : z;
    }
}

// dA = dZ W (dZ: B x O, W: O x I); times gelu'(Zprev) when Zprev is given.
__global__ __launch_bounds__(256) void linear_bwd_data_kernel(const float* __restrict__ dZ, int B, int O,
                                                              const float* __restrict__ W, int I,
                                                              const float* __restrict__ Zprev,
                                                              float* __restrict__ dA) {
    __shared__ float Ds[ML_TB][ML_KC + 1];
    __shared__ float Ws[ML_KC][ML_TO + 1];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * ML_TO, b0 = blockIdx.y * ML_TB;
    const int il = tid % ML_TO, bg = tid / ML_TO;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < O; k0 += ML_KC) {
        for (int e = tid; e < ML_TB * ML_KC; e += 256) {
            const int r = e / ML_KC, c = e % ML_KC;
            Ds[r][c] = (b0 + r < B && k0 + c < O) ? dZ[(size_t)(b0 + r) * O + k0 + c] : 0.f;
        }
        for (int e = tid; e < ML_KC * ML_TO; e += 256) {
            const int r = e / ML_TO, c = e % ML_TO;
            Ws[r][c] = (k0 + r < O && i0 + c < I) ? W[(size_t)(k0 + r) * I + i0 + c] : 0.f;
        }
        __syncthreads();
#pragma unroll 8
        for (int c = 0; c < ML_KC; ++c) {
            const float w = Ws[c][il];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = fmaf(Ds[bg * 4 + q][c], w, acc[q]);
        }
        __syncthreads();
    }
    const int i = i0 + il;
    if (i >= I) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int b = b0 + bg * 4 + q;
        if (b >= B) continue;
        float v = acc[q];
        if (Zprev) v *= gelu_grad_f(Zprev[(size_t)b * I + i]);
        dA[(size_t)b * I + i] = v;
    }
}

// gW = dZ^T A (O x I), gb = column sums of dZ; the batch is summed in order.
__global__ void linear_bwd_weight_kernel(const float* __restrict__ dZ, const float* __restrict__ A, int B, int O,
                                         int I, float* __restrict__ gW, float* __restrict__ gb) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nw = (size_t)O * I;
    if (e < nw) {
        const int o = (int)(e / I), i = (int)(e % I);
        float acc = 0.f;
        for (int b = 0; b < B; ++b) acc = fmaf(dZ[(size_t)b * O + o], A[(size_t)b * I + i], acc);
        gW[e] = acc;
    } else if (e < nw + O) {
        const int o = (int)(e - nw);
        float acc = 0.f;
        for (int b = 0; b < B; ++b) acc += dZ[(size_t)b * O + o];
        gb[o] = acc;
    }
}

// ---------------------------------------------------------------------------
// bfloat16 matrix-core products.  C (M x N) = sum_k a(m, k) b(k, n) with
//   MM_FWD:         a = A (B x I), b(k, n) = W[n][k]; M = B, N = O, K = I;
//                   epilogue z = C + bias, Z = z, Aout = gelu(z) or z
//   MM_BWD_DATA:    a = dZ (B x O), b(k, n) = W[k][n]; M = B, N = I, K = O;
//                   epilogue dA = C (times gelu'(Zprev) when given)
//   MM_BWD_WEIGHT:  a(m, k) = dZ[k][m], b(k, n) = A[k][n]; M = O, N = I, K = B;
//                   epilogue gW = C
// A workgroup (4 waves) owns a 32 x 64 tile of C; wave w a 16 x 32 strip
// (two 16 x 16 MFMA blocks).  Per 32-wide k chunk the operands are staged in
// LDS as bfloat16, k contiguous per row of a and per column of b, so that a
// lane's 8 k values are one 16-byte read: lane l supplies row (column) l % 16
// and k values 8 (l / 16) .. 8 (l / 16) + 7 of the chunk, for a and b alike.
enum { MM_FWD = 0, MM_BWD_DATA = 1, MM_BWD_WEIGHT = 2 };
constexpr int MM_TM = 32, MM_TN = 64, MM_KC = 32, MM_LD = MM_KC + 8;

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef short s16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

struct MmArgs {
    const float* a;
    const void* b;          // bfloat16 weights (MM_FWD, MM_BWD_DATA) or FP32 A (MM_BWD_WEIGHT)
    const float* bias;      // MM_FWD
    const float* zprev;     // MM_BWD_DATA, may be null
    float* out;             // Z, dA or gW
    float* out2;            // MM_FWD: the activation
    int M, N, K, act;
};

__device__ __forceinline__ bf16x8_t lds_bf16x8(const bf16_t* p) {
    return __builtin_bit_cast(bf16x8_t, *(const s16x8_t*)p);
}

template <int MODE>
__global__ __launch_bounds__(256) void mlp_mfma_kernel(MmArgs g) {
    constexpr bool BSPLIT = MODE == MM_BWD_WEIGHT;   // b is FP32 too: split it
    __shared__ __align__(16) bf16_t Ah[MM_TM * MM_LD], Al[MM_TM * MM_LD];
    __shared__ __align__(16) bf16_t Bh[MM_TN * MM_LD], Bl[BSPLIT ? MM_TN * MM_LD : 8];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * MM_TM, n0 = blockIdx.x * MM_TN;
    const int wm = (w & 1) * 16, wn = (w >> 1) * 32;
    const int r = lane & 15, kg = (lane >> 4) * 8;
    const float* A = g.a;
    f32x4_t acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    for (int k0 = 0; k0 < g.K; k0 += MM_KC) {
        // a: k contiguous in memory except for the weight gradient (m contiguous)
        for (int e = tid; e < MM_TM * MM_KC; e += 256) {
            const int mm = MODE == MM_BWD_WEIGHT ? e % MM_TM : e / MM_KC;
            const int kk = MODE == MM_BWD_WEIGHT ? e / MM_TM : e % MM_KC;
            const int m = m0 + mm, k = k0 + kk;
            float v = 0.f;
            if (m < g.M && k < g.K) v = MODE == MM_BWD_WEIGHT ? A[(size_t)k * g.M + m] : A[(size_t)m * g.K + k];
            const bf16_t h = f_to_bf16(v);
            Ah[mm * MM_LD + kk] = h;
            Al[mm * MM_LD + kk] = f_to_bf16(v - bf16_to_f(h));
        }
        // b: k contiguous for the forward product, n contiguous otherwise
        for (int e = tid; e < MM_TN * MM_KC; e += 256) {
            const int nn = MODE == MM_FWD ? e / MM_KC : e % MM_TN;
            const int kk = MODE == MM_FWD ? e % MM_KC : e / MM_TN;
            const int n = n0 + nn, k = k0 + kk;
            const bool in = n < g.N && k < g.K;
            if (MODE == MM_BWD_WEIGHT) {
                const float v = in ? ((const float*)g.b)[(size_t)k * g.N + n] : 0.f;
                const bf16_t h = f_to_bf16(v);
                Bh[nn * MM_LD + kk] = h;
                Bl[nn * MM_LD + kk] = f_to_bf16(v - bf16_to_f(h));
            } else {
                const bf16_t* W = (const bf16_t*)g.b;
                Bh[nn * MM_LD + kk] =
                    in ? (MODE == MM_FWD ? W[(size_t)n * g.K + k] : W[(size_t)k * g.N + n]) : (bf16_t)0;
            }
        }
        __syncthreads();
        const bf16x8_t ah = lds_bf16x8(&Ah[(wm + r) * MM_LD + kg]);
        const bf16x8_t al = lds_bf16x8(&Al[(wm + r) * MM_LD + kg]);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const bf16x8_t bh = lds_bf16x8(&Bh[(wn + j * 16 + r) * MM_LD + kg]);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[j], 0, 0, 0);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[j], 0, 0, 0);
            if (BSPLIT) {
                const bf16x8_t bl = lds_bf16x8(&Bl[(wn + j * 16 + r) * MM_LD + kg]);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // lane l holds rows 4 (l / 16) + i, column l % 16 of each 16 x 16 block
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int n = n0 + wn + j * 16 + r;
        if (n >= g.N) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = m0 + wm + (lane >> 4) * 4 + i;
            if (m >= g.M) continue;
            const size_t o = (size_t)m * g.N + n;
            float v = acc[j][i];
            if (MODE == MM_FWD) {
                v += g.bias[n];
                g.out[o] = v;
                g.out2[o] = g.act ? gelu_f(v) : v;
            } else if (MODE == MM_BWD_DATA) {
                if (g.zprev) v *= gelu_grad_f(g.zprev[o]);
                g.out[o] = v;
            } else {
                g.out[o] = v;
            }
        }
    }
}

// gb = column sums of dZ (B x O), the batch summed in order
__global__ void bias_grad_kernel(const float* __restrict__ dZ, int B, int O, float* __restrict__ gb) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= O) return;
    float acc = 0.f;
    for (int b = 0; b < B; ++b) acc += dZ[(size_t)b * O + o];
    gb[o] = acc;
}

template <int MODE>
static hipError_t launch_mm(const MmArgs& g, hipStream_t s) {
    dim3 grid((g.N + MM_TN - 1) / MM_TN, (g.M + MM_TM - 1) / MM_TM);
    hipLaunchKernelGGL(mlp_mfma_kernel<MODE>, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// dY = 2 (Y - T) / (B O); loss = mean (Y - T)^2 (one workgroup, fixed order).
__global__ __launch_bounds__(1024) void mse_kernel(const float* __restrict__ Y, const float* __restrict__ T, int count,
                                                   float* __restrict__ dY, double* __restrict__ loss) {
    __shared__ double red[1024];
    const int tid = threadIdx.x;
    const float sc = 2.0f / (float)count;
    double s = 0.0;
    for (int e = tid; e < count; e += 1024) {
        const float d = Y[e] - T[e];
        dY[e] = sc * d;
        s += (double)d * (double)d;
    }
    red[tid] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) *loss = red[0] / (double)count;
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, bf16_t* __restrict__ pb, size_t n, float lr, float b1, float b2,
                            float eps, float bc1, float bc2) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = pi;
    pb[i] = f_to_bf16(pi);
}

__global__ void to_bf16_kernel(const float* __restrict__ p, bf16_t* __restrict__ pb, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) pb[i] = f_to_bf16(p[i]);
}

// ---------------------------------------------------------------------------

namespace {
inline uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
}  // namespace

int Mlp::init(int nin_, int nh_, int nl_, int nout_, int bmax_, bool bf16_, uint64_t seed) {
    nin = nin_; nh = nh_; nl = nl_; nout = nout_; bmax = bmax_; bf16 = bf16_; t = 0;
    dims.clear();
    dims.push_back(nin);
    for (int l = 0; l < nl; ++l) dims.push_back(nh);
    dims.push_back(nout);
    nparam = 0;
    woff.clear();
    for (size_t l = 0; l + 1 < dims.size(); ++l) {
        woff.push_back(nparam);
        nparam += (size_t)dims[l + 1] * dims[l] + dims[l + 1];
    }
    // activations: per layer its input A_l (B x dims[l]) and pre-activation Z_l (B x dims[l+1]),
    // plus the network output and two gradient buffers of the widest layer
    size_t wmax = 0, acts = 0;
    for (size_t l = 0; l < dims.size(); ++l) {
        wmax = std::max<size_t>(wmax, dims[l]);
        acts += dims[l];
    }
    const size_t fl = (size_t)bmax * (2 * acts + 2 * wmax);
    hipError_t e;
    if ((e = hipMalloc(&p, nparam * 4)) != hipSuccess || (e = hipMalloc(&g, nparam * 4)) != hipSuccess ||
        (e = hipMalloc(&m, nparam * 4)) != hipSuccess || (e = hipMalloc(&v, nparam * 4)) != hipSuccess ||
        (e = hipMalloc(&pb, nparam * 2)) != hipSuccess || (e = hipMalloc(&work, fl * 4)) != hipSuccess ||
        (e = hipMalloc(&dloss, sizeof(double))) != hipSuccess)
        return e == hipErrorOutOfMemory ? MFD_ENOMEM : MFD_EDEVICE;
    return randomize(seed, nullptr);
}

int Mlp::randomize(uint64_t seed, hipStream_t s) {
    // uniform(-s, s), s = sqrt(6 / (in + out)) (Glorot); biases zero; the output
    // layer starts at zero so that the untrained network predicts no change
    std::vector<float> h(nparam, 0.0f);
    uint64_t st = seed * 0x2545F4914F6CDD1Dull + 12345;
    for (size_t l = 0; l + 1 < dims.size(); ++l) {
        if (l + 2 == dims.size()) break;
        const double sc = std::sqrt(6.0 / (dims[l] + dims[l + 1]));
        const size_t nw = (size_t)dims[l + 1] * dims[l];
        for (size_t i = 0; i < nw; ++i) {
            const double u = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
            h[woff[l] + i] = (float)((2.0 * u - 1.0) * sc);
        }
    }
    return set_params(h.data(), s);
}

int Mlp::set_params(const float* host, hipStream_t s) {
    hipError_t e;
    if ((e = hipMemcpyAsync(p, host, nparam * 4, hipMemcpyHostToDevice, s)) != hipSuccess) return MFD_EDEVICE;
    if ((e = hipMemsetAsync(m, 0, nparam * 4, s)) != hipSuccess) return MFD_EDEVICE;
    if ((e = hipMemsetAsync(v, 0, nparam * 4, s)) != hipSuccess) return MFD_EDEVICE;
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((nparam + 255) / 256)), dim3(256), 0, s, p, (bf16_t*)pb,
                       nparam);
    if (hipGetLastError() != hipSuccess) return MFD_EDEVICE;
    t = 0;
    return hipStreamSynchronize(s) == hipSuccess ? MFD_OK : MFD_EDEVICE;
}

void Mlp::release() {
    hipFree(p); hipFree(g); hipFree(m); hipFree(v); hipFree(pb); hipFree(work); hipFree(dloss);
    p = g = m = v = nullptr;
    pb = nullptr;
    work = nullptr;
    dloss = nullptr;
}

// layout of work: A_0 .. A_L (inputs, A_0 = x copy not needed: x is read in
// place), Z_0 .. Z_L, then dA, dB ping-pong buffers
float* Mlp::act_in(int l) const {
    size_t off = 0;
    for (int q = 0; q < l; ++q) off += (size_t)bmax * dims[q];
    return work + off;
}
float* Mlp::pre(int l) const {
    size_t off = 0;
    for (size_t q = 0; q < dims.size(); ++q) off += (size_t)bmax * dims[q];
    for (int q = 0; q < l; ++q) off += (size_t)bmax * dims[q + 1];
    return work + off;
}
float* Mlp::grad_buf(int which) const {
    size_t off = 0, wmax = 0;
    for (size_t q = 0; q < dims.size(); ++q) {
        off += 2 * (size_t)bmax * dims[q];
        wmax = std::max<size_t>(wmax, dims[q]);
    }
    return work + off + (size_t)which * bmax * wmax;
}

static hipError_t run_fwd(const Mlp& net, int B, const float* X, float* Y, hipStream_t s) {
    const int L = (int)net.dims.size() - 1;
    const float* a = X;
    for (int l = 0; l < L; ++l) {
        const int I = net.dims[l], O = net.dims[l + 1];
        const size_t wo = net.woff[l];
        float* out = (l == L - 1) ? Y : net.act_in(l + 1);
        const int act = l < L - 1 ? 1 : 0;
        hipError_t e;
        if (net.bf16) {
            MmArgs g{a, (const bf16_t*)net.pb + wo, net.p + wo + (size_t)O * I, nullptr, net.pre(l), out, B, O, I, act};
            e = launch_mm<MM_FWD>(g, s);
        } else {
            dim3 grid((O + ML_TO - 1) / ML_TO, (B + ML_TB - 1) / ML_TB);
            hipLaunchKernelGGL(linear_fwd_kernel, grid, dim3(256), 0, s, a, B, I, net.p + wo,
                               net.p + wo + (size_t)O * I, O, act, net.pre(l), out);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return e;
        a = out;
    }
    return hipSuccess;
}

hipError_t Mlp::forward(int B, const float* X, float* Y, hipStream_t s) { return run_fwd(*this, B, X, Y, s); }

static hipError_t run_bwd(const Mlp& net, int B, const float* X, const float* dY, hipStream_t s) {
    const int L = (int)net.dims.size() - 1;
    const float* dZ = dY;
    int which = 0;
    for (int l = L - 1; l >= 0; --l) {
        const int I = net.dims[l], O = net.dims[l + 1];
        const size_t wo = net.woff[l];
        const float* a_in = (l == 0) ? X : net.act_in(l);
        hipError_t e;
        if (net.bf16) {
            MmArgs g{dZ, a_in, nullptr, nullptr, net.g + wo, nullptr, O, I, B, 0};
            if ((e = launch_mm<MM_BWD_WEIGHT>(g, s)) != hipSuccess) return e;
            hipLaunchKernelGGL(bias_grad_kernel, dim3((O + 255) / 256), dim3(256), 0, s, dZ, B, O,
                               net.g + wo + (size_t)O * I);
        } else {
            const size_t nw = (size_t)O * I + O;
            hipLaunchKernelGGL(linear_bwd_weight_kernel, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, dZ,
                               a_in, B, O, I, net.g + wo, net.g + wo + (size_t)O * I);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (l == 0) break;
        float* dA = net.grad_buf(which);
        which ^= 1;
        if (net.bf16) {
            MmArgs g{dZ, (const bf16_t*)net.pb + wo, nullptr, net.pre(l - 1), dA, nullptr, B, I, O, 0};
            e = launch_mm<MM_BWD_DATA>(g, s);
        } else {
            dim3 grid((I + ML_TO - 1) / ML_TO, (B + ML_TB - 1) / ML_TB);
            hipLaunchKernelGGL(linear_bwd_data_kernel, grid, dim3(256), 0, s, dZ, B, O, net.p + wo, I,
                               net.pre(l - 1), dA);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return e;
        dZ = dA;
    }
    return hipSuccess;
}

hipError_t Mlp::loss_grad(int B, const float* X, const float* T, hipStream_t s) {
    // the output goes to the last activation slot and dY to gradient buffer 1:
    // the first backward layer reads dY and writes its dA to buffer 0
    float* Y = act_in((int)dims.size() - 1);
    float* dY = grad_buf(1);
    hipError_t e = forward(B, X, Y, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(1024), 0, s, Y, T, B * nout, dY, dloss);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return run_bwd(*this, B, X, dY, s);
}

hipError_t Mlp::adam(float lr, hipStream_t s) {
    ++t;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float bc1 = 1.0f - (float)std::pow(0.9, t), bc2 = 1.0f - (float)std::pow(0.999, t);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((nparam + 255) / 256)), dim3(256), 0, s, p, g, m, v, (bf16_t*)pb,
                       nparam, lr, b1, b2, eps, bc1, bc2);
    return hipGetLastError();
}

}  // namespace mfd
