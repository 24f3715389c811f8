// Register-resident passes of the FFT solve (Section 5.2, Alg 5.1) for FP32
// storage on cubic order-2 contexts of N = 16, 32 or 64: the same three
// passes as fft.hip (x-y plane transform, z transform with the 3 x 3 symbol
// solve, inverse plane transform), with every 1-D transform of length N held
// in one lane's registers.
//
//   plane pass:  one wave per (band, component, z) plane.  The plane is read
//     coalesced into LDS (rows padded to N + 1), lane l takes row l into its
//     registers and transforms it along x, writes it back, takes column l and
//     transforms it along y; column l then goes to HBM as N coalesced stores
//     (lane l = x).  No barrier: one wave per workgroup.
//   z pass:  one wave per (band, y, run of 16 x): lane (c, x) holds the z
//     column of component c at x (48 of 64 lanes), transforms it, forms the
//     3 x 3 solve at every frequency with the other two components fetched
//     across lanes, transforms back and stores.
//
// The transforms are radix-2 decimation in frequency, fully unrolled, output
// in bit-reversed register order (relabelled at compile time); twiddles
// exp(-2 pi i m / N) come from the context's table through scalar loads.
#include "common.h"
#include "internal.h"

namespace mfd {
namespace {

constexpr int bitrev(int x, int bits) {
    int r = 0;
    for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1) << (bits - 1 - i);
    return r;
}
constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// In-register DFT of length N (power of two): v[bitrev(k)] = sum_r v[r] w^(+-rk)
template <int N, bool INV>
__device__ __forceinline__ void fft_reg(float2 (&v)[N], const float2* __restrict__ tw) {
#pragma unroll
    for (int len = N; len >= 2; len >>= 1) {
        const int half = len >> 1;
#pragma unroll
        for (int j = 0; j < half; ++j) {
            float2 w = tw[j * (N / len)];
            if (INV) w.y = -w.y;
#pragma unroll
            for (int st = 0; st < N; st += len) {
                const float2 a = v[st + j], b = v[st + j + half];
                v[st + j] = cadd(a, b);
                v[st + j + half] = j ? cmul(csub(a, b), w) : csub(a, b);
            }
        }
    }
}

// The same DFT by decimation in time: input in bit-reversed register order
// (v[bitrev(k)] = x_k), output in natural order.
template <int N, bool INV>
__device__ __forceinline__ void fft_reg_dit(float2 (&v)[N], const float2* __restrict__ tw) {
#pragma unroll
    for (int len = 2; len <= N; len <<= 1) {
        const int half = len >> 1;
#pragma unroll
        for (int j = 0; j < half; ++j) {
            float2 w = tw[j * (N / len)];
            if (INV) w.y = -w.y;
#pragma unroll
            for (int st = 0; st < N; st += len) {
                const float2 a = v[st + j], b = j ? cmul(v[st + j + half], w) : v[st + j + half];
                v[st + j] = cadd(a, b);
                v[st + j + half] = csub(a, b);
            }
        }
    }
}

// forward (INV false) or inverse plane transform along x and y
template <int N, bool INV>
__global__ __launch_bounds__(64) void fft_plane_reg_kernel(const float2* __restrict__ in, float2* __restrict__ out,
                                                           const float2* __restrict__ tw, FieldList fl) {
    constexpr int LD = N + 1;
    constexpr int BITS = ilog2(N);
    __shared__ float2 buf[N * LD];
    const int lane = threadIdx.x;
    const size_t plane = (size_t)fl(blockIdx.x / (3 * N)) * 3 * N + blockIdx.x % (3 * N);
    const float2* src = in + plane * N * N;
    float2* dst = out + plane * N * N;
    float2 v[N];
    if (!INV) {
        // coalesced load into LDS; lane l then takes row l
        for (int i = lane; i < N * N; i += 64) buf[(i / N) * LD + i % N] = src[i];
        __builtin_amdgcn_wave_barrier();
        if (lane < N) {
#pragma unroll
            for (int x = 0; x < N; ++x) v[x] = buf[lane * LD + x];
            fft_reg<N, false>(v, tw);
#pragma unroll
            for (int k = 0; k < N; ++k) buf[lane * LD + k] = v[bitrev(k, BITS)];
        }
        __builtin_amdgcn_wave_barrier();
        // lane l = x takes column l, transforms along y, stores coalesced
        if (lane < N) {
#pragma unroll
            for (int y = 0; y < N; ++y) v[y] = buf[y * LD + lane];
            fft_reg<N, false>(v, tw);
#pragma unroll
            for (int k = 0; k < N; ++k) dst[(size_t)k * N + lane] = v[bitrev(k, BITS)];
        }
    } else {
        // lane l = x loads column l coalesced, transforms along y
        if (lane < N) {
#pragma unroll
            for (int y = 0; y < N; ++y) v[y] = src[(size_t)y * N + lane];
            fft_reg<N, true>(v, tw);
#pragma unroll
            for (int k = 0; k < N; ++k) buf[k * LD + lane] = v[bitrev(k, BITS)];
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < N) {
#pragma unroll
            for (int x = 0; x < N; ++x) v[x] = buf[lane * LD + x];
            fft_reg<N, true>(v, tw);
#pragma unroll
            for (int k = 0; k < N; ++k) buf[lane * LD + k] = v[bitrev(k, BITS)];
        }
        __builtin_amdgcn_wave_barrier();
        for (int i = lane; i < N * N; i += 64) dst[i] = buf[(i / N) * LD + i % N];
    }
}

struct RegSolveArgs {
    const float2* in;
    float2* out;
    const float2* tw;
    float inv_h, half_k[3], gm1, gamma, shift, scale;
    FieldList fl;
};

// z transform, 3 x 3 symbol solve, inverse z transform; XR = 16 x positions
// per wave, lane = c * 16 + x (c the component), lanes 48..63 idle
template <int N>
__global__ __launch_bounds__(64) void fft_zsolve_reg_kernel(RegSolveArgs a) {
    constexpr int XR = N < 16 ? N : 16;
    constexpr int NXR = N / XR;
    constexpr int BITS = ilog2(N);
    const int lane = threadIdx.x;
    const int c = lane / XR, xl = lane % XR;
    const bool act = c < 3;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int x0 = (bid % NXR) * XR;
    const int y = (bid / NXR) % N;
    const int band = a.fl(bid / (NXR * N));
    const size_t NN = (size_t)N * N, N3 = NN * N;
    const int x = x0 + xl;
    const size_t base = (size_t)band * 3 * N3 + (size_t)(act ? c : 0) * N3 + (size_t)y * N + x;
    float2 v[N];
#pragma unroll
    for (int z = 0; z < N; ++z) v[z] = act ? a.in[base + (size_t)z * NN] : mk<float2>(0.f, 0.f);
    fft_reg<N, false>(v, a.tw);
    // symbols of D_1 at px = x and D_2 at y (this lane's), D_3 at each pz
    auto sym = [&](int p, int axis) {
        float2 e = a.tw[p];
        e.y = -e.y;   // e^{i theta}
        return mk<float2>((e.x - 1.f) * a.inv_h - a.half_k[axis] * e.y, e.y * a.inv_h + a.half_k[axis] * (1.f + e.x));
    };
    const float2 d1 = sym(x, 0), d2 = sym(y, 1);
    const int src1 = ((c + 1) % 3) * XR + xl, src2 = ((c + 2) % 3) * XR + xl;   // the other components' lanes
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int pz = k;
        const float2 mine = v[bitrev(k, BITS)];
        // the other two components at the same (x, pz)
        const float2 o1 = mk<float2>(__shfl(mine.x, src1), __shfl(mine.y, src1));
        const float2 o2 = mk<float2>(__shfl(mine.x, src2), __shfl(mine.y, src2));
        // component 0, 1, 2 at (x, pz): this lane's, the next one's, the one after
        const float2 r0 = c == 0 ? mine : c == 1 ? o2 : o1;
        const float2 r1 = c == 0 ? o1 : c == 1 ? mine : o2;
        const float2 r2 = c == 0 ? o2 : c == 1 ? o1 : mine;
        const float2 d3 = sym(pz, 2);
        const float s = cabs2(d1) + cabs2(d2) + cabs2(d3);
        float2 dr = cmul(d1, r0);
        dr = cfma(dr, d2, r1);
        dr = cfma(dr, d3, r2);
        dr = cscale(dr, a.gm1 / (a.gamma * s + a.shift));
        const float2 dc = c == 0 ? d1 : c == 1 ? d2 : d3;
        v[bitrev(k, BITS)] = cscale(csub(mine, cmulc(dc, dr)), a.scale / (s + a.shift));
    }
    // inverse z transform: the frequencies sit in bit-reversed register
    // order, which decimation in time takes as input
    fft_reg_dit<N, true>(v, a.tw);
    if (act) {
        float2* dst = a.out + base;
#pragma unroll
        for (int z = 0; z < N; ++z) dst[(size_t)z * NN] = v[z];
    }
}

template <int N>
hipError_t reg_precond_n(const OpParams& p, int nb, const void* Rin, void* Tout, const void* tw, hipStream_t s,
                         const FieldList& fl) {
    const int nplanes = nb * 3 * N;
    hipLaunchKernelGGL((fft_plane_reg_kernel<N, false>), dim3(nplanes), dim3(64), 0, s, (const float2*)Rin,
                       (float2*)Tout, (const float2*)tw, fl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    RegSolveArgs a;
    a.in = (const float2*)Tout;
    a.out = (float2*)Tout;
    a.tw = (const float2*)tw;
    a.inv_h = (float)(1.0 / p.h);
    for (int i = 0; i < 3; ++i) a.half_k[i] = (float)(0.5 * p.k[i]);
    a.gm1 = (float)(p.gamma - 1.0);
    a.gamma = (float)p.gamma;
    a.shift = (float)p.shift;
    a.scale = (float)(1.0 / ((double)N * N * N));
    a.fl = fl;
    constexpr int XR = N < 16 ? N : 16;
    hipLaunchKernelGGL(fft_zsolve_reg_kernel<N>, dim3(nb * N * (N / XR)), dim3(64), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((fft_plane_reg_kernel<N, true>), dim3(nplanes), dim3(64), 0, s, (const float2*)Tout,
                       (float2*)Tout, (const float2*)tw, fl);
    return hipGetLastError();
}

}  // namespace

bool reg_precond_ok(const OpParams& p) {
    return !p.lattice && p.order == 2 && (p.N == 16 || p.N == 32 || p.N == 64);
}

hipError_t launch_precond_reg(const OpParams& p, int nb, const void* Rin, void* Tout, const void* tw, hipStream_t s,
                              const FieldList& fl) {
    if (fl.on && nb > 32) return hipErrorInvalidValue;
    switch (p.N) {
        case 16: return reg_precond_n<16>(p, nb, Rin, Tout, tw, s, fl);
        case 32: return reg_precond_n<32>(p, nb, Rin, Tout, tw, s, fl);
        case 64: return reg_precond_n<64>(p, nb, Rin, Tout, tw, s, fl);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mfd
