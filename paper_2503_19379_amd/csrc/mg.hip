// Multigrid solve of the preconditioner system (Section 5.3; Alg 5.2), the
// paper's second preconditioner solver beside the FFT solve of Alg 5.1.
//
// (P + c) x = f, P = A A' + gamma B'B, is split by the distributive form of
// Section 5.3 into scalar problems with the cell Laplacian L_k = B B' of
// Cor 4.4 (A A' + B'B = diag(L_k, L_k, L_k), and B A = 0):
//     y = (L_k + c)^-1 f           three scalar solves per field,
//     q = -(L_k + c/gamma)^-1 ((gamma - 1)/gamma) B y,
//     x = y + B' q.
// Each scalar solve is a fixed number of V-cycles (Alg 5.2) from a zero
// guess on the hierarchy N, N/2, ... (rediscretised L_k + sigma, h doubled,
// halving while N is even and above 4):
//   pre-smoothing n1 times, residual, restriction (cell-centred full
//   weighting), the cycle on the coarser grid, prolongation (trilinear, cell
//   centred) of its result added as the correction, post-smoothing n2 times;
//   on the coarsest grid (at most 5^3 points) the exact solve, a periodic
//   convolution with the inverse of the stencil's symbol.
// Smoothing step: x <- x + (L U)^-1 (b - A x), with L U the ILU(0) of the
// constant 7-point stencil A = (a; cm_i at -e_i; cp_i at +e_i): L = d I +
// lower couplings, U = I + upper couplings / d, d = a - sum_i cm_i cp_i / d.
// Each triangular factor is inverted approximately by `sweeps` Jacobi sweeps
// (SAIT's Jacobi iteration, applied to the vector), so every step is a
// stencil pass over the grid: no triangular solve.
//
// Every kernel here is a bandwidth-bound pass over FP64 complex grids, one
// thread per (field, cell), fields batched in one launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "common.h"
#include "internal.h"

namespace mfd {

using C128 = double2;

// Constant 7-point stencil of L_k + sigma on one level (FP64 complex).
struct MGStencil {
    double a;           // centre (real: L_k is Hermitian)
    C128 cm[3], cp[3];  // couplings to -e_i and +e_i, axis i = x, y, z
    double d;           // diagonal of the ILU factors
    int N;
};

namespace {

__device__ __forceinline__ size_t cell(int x, int y, int z, int N) { return (size_t)x + (size_t)N * (y + (size_t)N * z); }

// A u at cell (x, y, z) of field f
__device__ __forceinline__ C128 apply_at(const C128* __restrict__ u, int x, int y, int z, const MGStencil& st) {
    const int N = st.N;
    const int xm = x ? x - 1 : N - 1, xp = x + 1 < N ? x + 1 : 0;
    const int ym = y ? y - 1 : N - 1, yp = y + 1 < N ? y + 1 : 0;
    const int zm = z ? z - 1 : N - 1, zp = z + 1 < N ? z + 1 : 0;
    C128 s = cscale(u[cell(x, y, z, N)], st.a);
    s = cfma(s, st.cm[0], u[cell(xm, y, z, N)]);
    s = cfma(s, st.cp[0], u[cell(xp, y, z, N)]);
    s = cfma(s, st.cm[1], u[cell(x, ym, z, N)]);
    s = cfma(s, st.cp[1], u[cell(x, yp, z, N)]);
    s = cfma(s, st.cm[2], u[cell(x, y, zm, N)]);
    s = cfma(s, st.cp[2], u[cell(x, y, zp, N)]);
    return s;
}

#define MG_LOOP(total)                                                                                            \
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (total); i += (size_t)gridDim.x * blockDim.x)

// r = b - A x; z1 = r / d.  x may be null (a zero guess: r = b).
__global__ void mg_residual_kernel(const C128* __restrict__ x, const C128* __restrict__ b, C128* __restrict__ r,
                                   C128* __restrict__ z1, size_t nf, MGStencil st) {
    const int N = st.N;
    const size_t n3 = (size_t)N * N * N;
    MG_LOOP(nf * n3) {
        const size_t f = i / n3, c = i % n3;
        const int xx = (int)(c % N), yy = (int)((c / N) % N), zz = (int)(c / ((size_t)N * N));
        C128 v = b[i];
        if (x) v = csub(v, apply_at(x + f * n3, xx, yy, zz, st));
        if (r) r[i] = v;
        if (z1) z1[i] = cscale(v, 1.0 / st.d);
    }
}

// Jacobi sweep on L z1 = r: z1n = (r - sum_i cm_i z1[-e_i]) / d
__global__ void mg_lsweep_kernel(const C128* __restrict__ r, const C128* __restrict__ z1, C128* __restrict__ z1n,
                                 size_t nf, MGStencil st) {
    const int N = st.N;
    const size_t n3 = (size_t)N * N * N;
    MG_LOOP(nf * n3) {
        const size_t f = i / n3, c = i % n3;
        const int x = (int)(c % N), y = (int)((c / N) % N), z = (int)(c / ((size_t)N * N));
        const C128* u = z1 + f * n3;
        C128 s = cmul(st.cm[0], u[cell(x ? x - 1 : N - 1, y, z, N)]);
        s = cfma(s, st.cm[1], u[cell(x, y ? y - 1 : N - 1, z, N)]);
        s = cfma(s, st.cm[2], u[cell(x, y, z ? z - 1 : N - 1, N)]);
        z1n[i] = cscale(csub(r[i], s), 1.0 / st.d);
    }
}

// Jacobi sweep on U z = z1: zn = z1 - sum_i (cp_i / d) z[+e_i]; with xacc,
// xacc += zn (the last sweep adds the correction to the iterate)
__global__ void mg_usweep_kernel(const C128* __restrict__ z1, const C128* __restrict__ z, C128* __restrict__ zn,
                                 C128* __restrict__ xacc, size_t nf, MGStencil st) {
    const int N = st.N;
    const size_t n3 = (size_t)N * N * N;
    const double id = 1.0 / st.d;
    MG_LOOP(nf * n3) {
        const size_t f = i / n3, c = i % n3;
        const int x = (int)(c % N), y = (int)((c / N) % N), zz = (int)(c / ((size_t)N * N));
        const C128* u = z + f * n3;
        C128 s = cmul(cscale(st.cp[0], id), u[cell(x + 1 < N ? x + 1 : 0, y, zz, N)]);
        s = cfma(s, cscale(st.cp[1], id), u[cell(x, y + 1 < N ? y + 1 : 0, zz, N)]);
        s = cfma(s, cscale(st.cp[2], id), u[cell(x, y, zz + 1 < N ? zz + 1 : 0, N)]);
        const C128 v = csub(z1[i], s);
        if (zn) zn[i] = v;
        if (xacc) xacc[i] = cadd(xacc[i], v);
    }
}

__global__ void mg_fill_zero_kernel(C128* __restrict__ x, size_t count) { MG_LOOP(count) x[i] = mk<C128>(0.0, 0.0); }

// x += z (smoothing with no Jacobi sweep: the correction is z1 = r / d)
__global__ void mg_add_kernel(const C128* __restrict__ z, C128* __restrict__ x, size_t count) {
    MG_LOOP(count) x[i] = cadd(x[i], z[i]);
}

// Full weighting: bc[I] = (1/8) sum over the 4 x 4 x 4 fine cells
// 2I-1 .. 2I+2 per axis with weights (1/4, 3/4, 3/4, 1/4): the adjoint of
// the trilinear prolongation divided by 8
__global__ void mg_restrict_kernel(const C128* __restrict__ r, C128* __restrict__ bc, int Nc, size_t nf) {
    const int N = 2 * Nc;
    const size_t nc3 = (size_t)Nc * Nc * Nc, n3 = (size_t)N * N * N;
    const double w[4] = {0.25, 0.75, 0.75, 0.25};
    MG_LOOP(nf * nc3) {
        const size_t f = i / nc3, c = i % nc3;
        const int X = (int)(c % Nc), Y = (int)((c / Nc) % Nc), Z = (int)(c / ((size_t)Nc * Nc));
        const C128* u = r + f * n3;
        C128 s = mk<C128>(0.0, 0.0);
        for (int a = 0; a < 4; ++a) {
            const int z = (2 * Z - 1 + a + N) % N;
            for (int b = 0; b < 4; ++b) {
                const int y = (2 * Y - 1 + b + N) % N;
                const double wzy = w[a] * w[b];
                for (int e = 0; e < 4; ++e) {
                    const int x = (2 * X - 1 + e + N) % N;
                    s = cadd(s, cscale(u[cell(x, y, z, N)], wzy * w[e]));
                }
            }
        }
        bc[i] = cscale(s, 0.125);
    }
}

// x[fine] += trilinear interpolation of the coarse xc: per axis, fine 2I
// takes 3/4 of coarse I and 1/4 of I-1, fine 2I+1 3/4 of I and 1/4 of I+1
__global__ void mg_prolong_kernel(const C128* __restrict__ xc, C128* __restrict__ x, int Nc, size_t nf) {
    const int N = 2 * Nc;
    const size_t nc3 = (size_t)Nc * Nc * Nc, n3 = (size_t)N * N * N;
    MG_LOOP(nf * n3) {
        const size_t f = i / n3, c = i % n3;
        const int fx = (int)(c % N), fy = (int)((c / N) % N), fz = (int)(c / ((size_t)N * N));
        int ix[2], iy[2], iz[2];
        double wx[2], wy[2], wz[2];
        auto pair = [&](int fi, int* idx, double* ww) {
            const int I = fi >> 1;
            idx[0] = I;
            ww[0] = 0.75;
            idx[1] = (fi & 1) ? (I + 1 < Nc ? I + 1 : 0) : (I ? I - 1 : Nc - 1);
            ww[1] = 0.25;
        };
        pair(fx, ix, wx);
        pair(fy, iy, wy);
        pair(fz, iz, wz);
        const C128* u = xc + f * nc3;
        C128 s = mk<C128>(0.0, 0.0);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int e = 0; e < 2; ++e)
                    s = cadd(s, cscale(u[cell(ix[e], iy[b], iz[a], Nc)], wz[a] * wy[b] * wx[e]));
        x[i] = cadd(x[i], s);
    }
}

// Coarsest grid: x[r] = sum_r' g[r - r'] b[r'] (periodic), g the inverse of
// the stencil's symbol transformed back (the exact inverse of the circulant)
__global__ void mg_coarse_kernel(const C128* __restrict__ g, const C128* __restrict__ b, C128* __restrict__ x, int Nc,
                                 size_t nf) {
    const size_t nc3 = (size_t)Nc * Nc * Nc;
    MG_LOOP(nf * nc3) {
        const size_t f = i / nc3, c = i % nc3;
        const int X = (int)(c % Nc), Y = (int)((c / Nc) % Nc), Z = (int)(c / ((size_t)Nc * Nc));
        const C128* u = b + f * nc3;
        C128 s = mk<C128>(0.0, 0.0);
        for (int z = 0; z < Nc; ++z)
            for (int y = 0; y < Nc; ++y)
                for (int x = 0; x < Nc; ++x) {
                    const int dx = (X - x + Nc) % Nc, dy = (Y - y + Nc) % Nc, dz = (Z - z + Nc) % Nc;
                    s = cfma(s, g[cell(dx, dy, dz, Nc)], u[cell(x, y, z, Nc)]);
                }
        x[i] = s;
    }
}

// g = scale (D_1 y_1 + D_2 y_2 + D_3 y_3) per band (cell scalar from face
// fields), D_i u[r] = (u[r+e_i] - u[r]) / h + i alpha_i (u[r+e_i] + u[r]) / 2
template <class S>
__global__ void mg_div_kernel(const C128* __restrict__ y, C128* __restrict__ g, int N, double inv_h, double a0, double a1,
                              double a2, double scale, size_t nb) {
    const size_t n3 = (size_t)N * N * N;
    const double al[3] = {a0, a1, a2};
    MG_LOOP(nb * n3) {
        const size_t bnd = i / n3, c = i % n3;
        const int x = (int)(c % N), yy = (int)((c / N) % N), z = (int)(c / ((size_t)N * N));
        const size_t nb_[3] = {cell(x + 1 < N ? x + 1 : 0, yy, z, N), cell(x, yy + 1 < N ? yy + 1 : 0, z, N),
                               cell(x, yy, z + 1 < N ? z + 1 : 0, N)};
        C128 s = mk<C128>(0.0, 0.0);
        for (int k = 0; k < 3; ++k) {
            const C128* u = y + (bnd * 3 + k) * n3;
            const C128 up = u[nb_[k]], u0 = u[c];
            // (up - u0)/h + i alpha (up + u0)/2
            const C128 df = cscale(csub(up, u0), inv_h);
            const C128 av = cscale(cadd(up, u0), 0.5 * al[k]);
            s = cadd(s, mk<C128>(df.x - av.y, df.y + av.x));
        }
        g[i] = cscale(s, scale);
    }
}

// T = y + B' q, (D_i' q)[r] = (q[r-e_i] - q[r]) / h - i alpha_i (q[r-e_i] + q[r]) / 2,
// written to the fields fl(b) of T (storage S)
template <class S>
__global__ void mg_assemble_kernel(const C128* __restrict__ y, const C128* __restrict__ q, S* __restrict__ T, int N,
                                   double inv_h, double a0, double a1, double a2, size_t nb, FieldList fl) {
    const size_t n3 = (size_t)N * N * N;
    const double al[3] = {a0, a1, a2};
    MG_LOOP(nb * 3 * n3) {
        const size_t bc = i / n3, c = i % n3;
        const size_t bnd = bc / 3;
        const int k = (int)(bc % 3);
        const int x = (int)(c % N), yy = (int)((c / N) % N), z = (int)(c / ((size_t)N * N));
        const size_t nm = k == 0 ? cell(x ? x - 1 : N - 1, yy, z, N)
                                 : k == 1 ? cell(x, yy ? yy - 1 : N - 1, z, N) : cell(x, yy, z ? z - 1 : N - 1, N);
        const C128* qb = q + bnd * n3;
        const C128 qm = qb[nm], q0 = qb[c];
        const C128 df = cscale(csub(qm, q0), inv_h);
        const C128 av = cscale(cadd(qm, q0), 0.5 * al[k]);
        // df - i av
        const C128 v = cadd(y[i], mk<C128>(df.x + av.y, df.y - av.x));
        T[((size_t)fl((int)bnd) * 3 + k) * n3 + c] = mk<S>(v.x, v.y);
    }
}

// gather the fields fl(b) of R (storage S) into the contiguous FP64 block y
template <class S>
__global__ void mg_gather_kernel(const S* __restrict__ R, C128* __restrict__ y, size_t n, size_t nb, FieldList fl) {
    MG_LOOP(nb * n) {
        const size_t b = i / n, c = i % n;
        const S v = R[(size_t)fl((int)b) * n + c];
        y[i] = mk<C128>((double)v.x, (double)v.y);
    }
}

unsigned blocks_for(size_t count) { return (unsigned)std::min<size_t>(4096, (count + 255) / 256); }

}  // namespace

// Per-caller work space of the multigrid solve: on each level, the iterate,
// right-hand side, residual and the two ping-pong pairs of the smoother, for
// `cap` scalar fields (level 0's iterate holds y, its right-hand side f and
// then the q problem's); q itself; and the coarsest-level inverses of the two
// scalar problems of the last Bloch vector (cached: a band solve applies the
// preconditioner at one k many times).
struct MGWork {
    int N = 0, cap = 0;
    std::vector<int> Ns;
    std::vector<C128*> x, b, r, z1a, z1b, za, zb;
    C128* q = nullptr;
    struct Coarse {
        double key[5] = {0, 0, 0, 0, -1};   // k, sigma, N
        C128* g = nullptr;
        std::vector<C128> host;
    } coarse[2];
    int next_slot = 0;
    void release() {
        for (auto* v : {&x, &b, &r, &z1a, &z1b, &za, &zb})
            for (C128* p : *v) (void)hipFree(p);
        x.clear(); b.clear(); r.clear(); z1a.clear(); z1b.clear(); za.clear(); zb.clear();
        (void)hipFree(q);
        q = nullptr;
        for (auto& c : coarse) {
            (void)hipFree(c.g);
            c.g = nullptr;
            c.key[4] = -1;
        }
        cap = 0;
    }
};

std::vector<int> mg_levels(int N) {
    std::vector<int> L{N};
    while (L.back() % 2 == 0 && L.back() > 4) L.push_back(L.back() / 2);
    return L;
}

bool mg_supported(int N) {
    if (N < 4) return false;
    return mg_levels(N).back() <= 5;
}

MGWork* mg_create() { return new MGWork(); }

void mg_destroy(MGWork* w) {
    if (!w) return;
    w->release();
    delete w;
}

// Stencil of L_k + sigma on a grid of n cells per axis (side L):
// D_i u[r] = a_i u[r+1] + b_i u[r] with a_i = 1/h + i alpha_i/2,
// b_i = -1/h + i alpha_i/2, so D_i D_i' has centre |a_i|^2 + |b_i|^2,
// coupling a_i conj(b_i) to +e_i and b_i conj(a_i) to -e_i.
static MGStencil make_stencil(int n, double L, const double k[3], double sigma) {
    MGStencil st;
    st.N = n;
    const double h = L / n;
    double a = sigma, s = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double ar = 1.0 / h, ai = 0.5 * k[i], br = -1.0 / h, bi = 0.5 * k[i];
        a += ar * ar + ai * ai + br * br + bi * bi;
        st.cp[i] = mk<C128>(ar * br + ai * bi, ai * br - ar * bi);   // a conj(b)
        st.cm[i] = mk<C128>(st.cp[i].x, -st.cp[i].y);
        s += st.cp[i].x * st.cp[i].x + st.cp[i].y * st.cp[i].y;     // cm_i cp_i = |cp_i|^2
    }
    st.a = a;
    st.d = 0.5 * (a + std::sqrt(a * a - 4.0 * s));
    return st;
}

// g[delta] = (1/n^3) sum_p e^{2 pi i p.delta / n} / s(p), s(p) = a + sum_i
// (cm_i e^{-i th_i} + cp_i e^{i th_i}) the stencil's symbol at frequency p
static void coarse_inverse(const MGStencil& st, std::vector<C128>& g) {
    const int n = st.N;
    const size_t n3 = (size_t)n * n * n;
    std::vector<C128> inv(n3);
    for (int pz = 0; pz < n; ++pz)
        for (int py = 0; py < n; ++py)
            for (int px = 0; px < n; ++px) {
                const int p[3] = {px, py, pz};
                double sr = st.a, si = 0.0;
                for (int i = 0; i < 3; ++i) {
                    const double th = 2.0 * M_PI * p[i] / n, c = std::cos(th), sn = std::sin(th);
                    sr += st.cm[i].x * c + st.cm[i].y * sn + st.cp[i].x * c - st.cp[i].y * sn;
                    si += st.cm[i].y * c - st.cm[i].x * sn + st.cp[i].y * c + st.cp[i].x * sn;
                }
                const double m = sr * sr + si * si;
                inv[px + (size_t)n * (py + (size_t)n * pz)] = mk<C128>(sr / m, -si / m);
            }
    g.assign(n3, mk<C128>(0.0, 0.0));
    for (int dz = 0; dz < n; ++dz)
        for (int dy = 0; dy < n; ++dy)
            for (int dx = 0; dx < n; ++dx) {
                double re = 0.0, im = 0.0;
                for (int pz = 0; pz < n; ++pz)
                    for (int py = 0; py < n; ++py)
                        for (int px = 0; px < n; ++px) {
                            const double th = 2.0 * M_PI * ((double)px * dx + (double)py * dy + (double)pz * dz) / n;
                            const C128 v = inv[px + (size_t)n * (py + (size_t)n * pz)];
                            const double c = std::cos(th), sn = std::sin(th);
                            re += v.x * c - v.y * sn;
                            im += v.x * sn + v.y * c;
                        }
                g[dx + (size_t)n * (dy + (size_t)n * dz)] = mk<C128>(re / n3, im / n3);
            }
}

static hipError_t ensure(MGWork* w, int N, int cap) {
    if (w->N == N && w->cap >= cap) return hipSuccess;
    w->release();
    w->N = N;
    w->Ns = mg_levels(N);
    const int nl = (int)w->Ns.size();
    auto get = [&](C128** p, size_t count) { return hipMalloc(p, count * sizeof(C128)); };
    hipError_t e;
    for (auto* v : {&w->x, &w->b, &w->r, &w->z1a, &w->z1b, &w->za, &w->zb}) v->assign(nl, nullptr);
    for (int l = 0; l < nl; ++l) {
        const size_t cnt = (size_t)cap * w->Ns[l] * w->Ns[l] * w->Ns[l];
        for (auto* v : {&w->x, &w->b, &w->r, &w->z1a, &w->z1b, &w->za, &w->zb})
            if ((e = get(&(*v)[l], cnt)) != hipSuccess) return e;
    }
    const int Nc = w->Ns.back();
    for (auto& c : w->coarse)
        if ((e = get(&c.g, (size_t)Nc * Nc * Nc)) != hipSuccess) return e;
    if ((e = get(&w->q, (size_t)((cap + 2) / 3) * N * N * N)) != hipSuccess) return e;
    w->cap = cap;
    return hipSuccess;
}

// One smoothing step on level l: x += (L U)^-1 (b - A x)
static hipError_t smooth_step(MGWork* w, int l, const MGStencil& st, C128* x, const C128* b, size_t nf, int sweeps,
                              hipStream_t s) {
    const size_t cnt = nf * (size_t)st.N * st.N * st.N;
    const unsigned nb = blocks_for(cnt);
    hipLaunchKernelGGL(mg_residual_kernel, dim3(nb), dim3(256), 0, s, x, b, w->r[l], w->z1a[l], nf, st);
    C128* z1 = w->z1a[l];
    C128* z1o = w->z1b[l];
    for (int k = 0; k < sweeps; ++k) {
        hipLaunchKernelGGL(mg_lsweep_kernel, dim3(nb), dim3(256), 0, s, w->r[l], z1, z1o, nf, st);
        std::swap(z1, z1o);
    }
    if (sweeps == 0) {
        hipLaunchKernelGGL(mg_add_kernel, dim3(nb), dim3(256), 0, s, z1, x, cnt);
        return hipGetLastError();
    }
    // U sweeps start from z = z1; the last one adds its result to x
    const C128* z = z1;
    C128* zout[2] = {w->za[l], w->zb[l]};
    for (int k = 0; k < sweeps; ++k) {
        const bool last = k + 1 == sweeps;
        C128* zn = last ? nullptr : zout[k & 1];
        hipLaunchKernelGGL(mg_usweep_kernel, dim3(nb), dim3(256), 0, s, z1, z, zn, last ? x : nullptr, nf, st);
        z = zn;
    }
    return hipGetLastError();
}

// V-cycle (Alg 5.2) on level l for nf fields: x the iterate, b the right-hand side
static hipError_t vcycle(MGWork* w, const std::vector<MGStencil>& H, const C128* g, int l, C128* x, const C128* b,
                         size_t nf, const MGOpts& o, hipStream_t s) {
    const int nl = (int)w->Ns.size();
    const MGStencil& st = H[l];
    const int N = st.N;
    const size_t cnt = nf * (size_t)N * N * N;
    if (l == nl - 1) {
        hipLaunchKernelGGL(mg_coarse_kernel, dim3(blocks_for(cnt)), dim3(256), 0, s, g, b, x, N, nf);
        return hipGetLastError();
    }
    hipError_t e;
    for (int k = 0; k < o.n1; ++k)
        if ((e = smooth_step(w, l, st, x, b, nf, o.sweeps, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(mg_residual_kernel, dim3(blocks_for(cnt)), dim3(256), 0, s, x, b, w->r[l], (C128*)nullptr, nf,
                       st);
    const int Nc = w->Ns[l + 1];
    const size_t cc = nf * (size_t)Nc * Nc * Nc;
    hipLaunchKernelGGL(mg_restrict_kernel, dim3(blocks_for(cc)), dim3(256), 0, s, w->r[l], w->b[l + 1], Nc, nf);
    // the coarse problem starts from zero: its first residual is its right-hand side
    hipLaunchKernelGGL(mg_fill_zero_kernel, dim3(blocks_for(cc)), dim3(256), 0, s, w->x[l + 1], cc);
    if ((e = vcycle(w, H, g, l + 1, w->x[l + 1], w->b[l + 1], nf, o, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(mg_prolong_kernel, dim3(blocks_for(cnt)), dim3(256), 0, s, w->x[l + 1], x, Nc, nf);
    for (int k = 0; k < o.n2; ++k)
        if ((e = smooth_step(w, l, st, x, b, nf, o.sweeps, s)) != hipSuccess) return e;
    return hipGetLastError();
}

// x = (L_k + sigma)^-1 b approximated by o.cycles V-cycles from zero
static hipError_t scalar_solve(MGWork* w, const OpParams& p, double sigma, C128* x, const C128* b, size_t nf,
                               const MGOpts& o, hipStream_t s) {
    std::vector<MGStencil> H;
    for (int n : w->Ns) H.push_back(make_stencil(n, p.L, p.k, sigma));
    const double key[5] = {p.k[0], p.k[1], p.k[2], sigma, (double)w->Ns.back()};
    MGWork::Coarse* slot = nullptr;
    for (auto& c : w->coarse)
        if (c.key[0] == key[0] && c.key[1] == key[1] && c.key[2] == key[2] && c.key[3] == key[3] &&
            c.key[4] == key[4])
            slot = &c;
    hipError_t e;
    if (!slot) {
        slot = &w->coarse[w->next_slot];
        w->next_slot ^= 1;
        coarse_inverse(H.back(), slot->host);
        if ((e = hipMemcpyAsync(slot->g, slot->host.data(), slot->host.size() * sizeof(C128), hipMemcpyHostToDevice,
                                s)) != hipSuccess)
            return e;
        // the host table is rewritten when the slot is reused: wait for the copy
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        for (int q = 0; q < 5; ++q) slot->key[q] = key[q];
    }
    const size_t cnt = nf * (size_t)p.N * p.N * p.N;
    hipLaunchKernelGGL(mg_fill_zero_kernel, dim3(blocks_for(cnt)), dim3(256), 0, s, x, cnt);
    for (int c = 0; c < o.cycles; ++c)
        if ((e = vcycle(w, H, slot->g, 0, x, b, nf, o, s)) != hipSuccess) return e;
    return hipGetLastError();
}

template <class S>
hipError_t launch_precond_mg(MGWork* w, const OpParams& p, const MGOpts& o, int nb, const void* Rin, void* Tout,
                             hipStream_t s, const FieldList& fl) {
    if (!w || p.order != 2 || p.lattice || !mg_supported(p.N)) return hipErrorInvalidValue;
    if (fl.on && nb > 32) return hipErrorInvalidValue;
    if (o.cycles < 1 || o.n1 < 0 || o.n2 < 0 || o.sweeps < 0) return hipErrorInvalidValue;
    if (nb <= 0) return hipSuccess;
    hipError_t e = ensure(w, p.N, 3 * nb);
    if (e != hipSuccess) return e;
    const size_t n3 = (size_t)p.N * p.N * p.N;
    // f: the 3 nb components of the right-hand side, as FP64 scalar fields
    hipLaunchKernelGGL(mg_gather_kernel<S>, dim3(blocks_for(3 * nb * n3)), dim3(256), 0, s, (const S*)Rin, w->b[0],
                       3 * n3, (size_t)nb, fl);
    // y = (L_k + c)^-1 f
    if ((e = scalar_solve(w, p, p.shift, w->x[0], w->b[0], 3 * (size_t)nb, o, s)) != hipSuccess) return e;
    // g = -((gamma - 1) / gamma) B y, then q = (L_k + c / gamma)^-1 g
    const double inv_h = 1.0 / p.h;
    hipLaunchKernelGGL(mg_div_kernel<S>, dim3(blocks_for(nb * n3)), dim3(256), 0, s, w->x[0], w->b[0], p.N, inv_h,
                       p.k[0], p.k[1], p.k[2], -(p.gamma - 1.0) / p.gamma, (size_t)nb);
    if ((e = scalar_solve(w, p, p.shift / p.gamma, w->q, w->b[0], (size_t)nb, o, s)) != hipSuccess) return e;
    // T = y + B' q
    hipLaunchKernelGGL(mg_assemble_kernel<S>, dim3(blocks_for(3 * nb * n3)), dim3(256), 0, s, w->x[0], w->q, (S*)Tout,
                       p.N, inv_h, p.k[0], p.k[1], p.k[2], (size_t)nb, fl);
    return hipGetLastError();
}

template hipError_t launch_precond_mg<double2>(MGWork*, const OpParams&, const MGOpts&, int, const void*, void*,
                                               hipStream_t, const FieldList&);
template hipError_t launch_precond_mg<float2>(MGWork*, const OpParams&, const MGOpts&, int, const void*, void*,
                                              hipStream_t, const FieldList&);

}  // namespace mfd
