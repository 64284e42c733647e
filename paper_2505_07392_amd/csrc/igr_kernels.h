// HIP kernels of the IGR right-hand side for gfx950 (wave64).
//
//   k_bc_state   ghost layers of the conserved state (periodic, zero-gradient
//                extrapolation, blended jet discs on the x-min face)
//   k_bc_sigma   ghost layers of Sigma (periodic or zero gradient)
//   k_source     b = alpha [tr((grad u)^2) + tr^2(grad u)], eq. (9) left side
//   k_jacobi     one Jacobi sweep of eq. (9)'s 7-point discretisation
//   (the fused reconstruction + LLF flux + divergence + SSP-RK3 stage kernel
//    is k_flux_tiled in igr_flux.h)
//   k_*_partial  deterministic FP64 block reductions (dt, sums, residual)
#pragma once

#include "igr_device.h"

namespace igr {

enum FluxMode { MODE_RHS = 0, MODE_STAGE1 = 1, MODE_STAGE2 = 2, MODE_STAGE3 = 3 };

// ---------------------------------------------------------------------------
// Boundary ghosts
// ---------------------------------------------------------------------------

// Face ghosts depend on interior cells only, so the faces of all three axes
// are filled by one launch: thread t is mapped to (axis, side, transverse
// cell), z faces first (their rows are contiguous), then y, then x.
// Returns false for threads past the last face.
__device__ __forceinline__ bool bc_face_of(const Geom& g, long long t, int& axis, long long& r) {
    const long long nz2 = 2LL * g.n[0] * g.n[1], ny2 = 2LL * g.n[0] * g.n[2], nx2 = 2LL * g.n[1] * g.n[2];
    if (t < nz2) {
        axis = 2;
        r = t;
    } else if (t < nz2 + ny2) {
        axis = 1;
        r = t - nz2;
    } else if (t < nz2 + ny2 + nx2) {
        axis = 0;
        r = t - nz2 - ny2;
    } else {
        return false;
    }
    return true;
}

inline long long bc_face_threads(const Geom& g) {
    return 2LL * g.n[0] * g.n[1] + 2LL * g.n[0] * g.n[2] + 2LL * g.n[1] * g.n[2];
}

// One thread per (transverse cell, side) of a face: writes the three ghost
// layers of the five fields.  Only face ghosts are written (edges and
// corners are never read by the axis-aligned stencils).
template <class T>
__global__ void k_bc_state(T* __restrict__ U, Geom g, const int* __restrict__ owner, const double* __restrict__ chi,
                           const double* __restrict__ jet) {
    using S = Storage<T>;
    using C = typename S::C;
    int axis;
    long long r;
    if (!bc_face_of(g, (long long)blockIdx.x * blockDim.x + threadIdx.x, axis, r)) return;
    const int a = axis == 0 ? 1 : 0;
    const int b = axis == 2 ? 1 : 2;
    const long long tot = (long long)g.n[a] * g.n[b];
    const int side = r >= tot;
    r -= side * tot;
    const int ia = int(r % g.n[a]);
    const int ib = int(r / g.n[a]);
    const long long base = (long long)(ia + G) * g.st[a] + (long long)(ib + G) * g.st[b];
    const int nd = g.n[axis];
    const int sd = g.st[axis];
    const int edge = side ? nd - 1 : 0;
    int q = -1;
    if (axis == 0 && side == 0 && owner != nullptr) q = owner[(long long)ib * g.n[1] + ia];
    for (int f = 0; f < 5; ++f) {
        T* F = U + f * g.fs + base;
        if (q >= 0) {
            const C c = C(chi[(long long)ib * g.n[1] + ia]);
            const C ext = S::load(F + (long long)(edge + G) * sd);
            const C v = c * C(jet[q * 5 + f]) + (C(1) - c) * ext;
            for (int l = 0; l < G; ++l) S::store(F + (long long)(-1 - l + G) * sd, v);
            continue;
        }
        for (int l = 0; l < G; ++l) {
            const int gi = side ? nd + l : -1 - l;
            int si = edge;
            if (g.periodic[axis]) si = ((gi % nd) + nd) % nd;
            F[(long long)(gi + G) * sd] = F[(long long)(si + G) * sd];
        }
    }
}

template <class T>
__global__ void k_bc_sigma(T* __restrict__ Sg, Geom g) {
    int axis;
    long long r;
    if (!bc_face_of(g, (long long)blockIdx.x * blockDim.x + threadIdx.x, axis, r)) return;
    const int a = axis == 0 ? 1 : 0;
    const int b = axis == 2 ? 1 : 2;
    const long long tot = (long long)g.n[a] * g.n[b];
    const int side = r >= tot;
    r -= side * tot;
    const int ia = int(r % g.n[a]);
    const int ib = int(r / g.n[a]);
    T* F = Sg + (long long)(ia + G) * g.st[a] + (long long)(ib + G) * g.st[b];
    const int nd = g.n[axis];
    const int sd = g.st[axis];
    const int edge = side ? nd - 1 : 0;
    for (int l = 0; l < G; ++l) {
        const int gi = side ? nd + l : -1 - l;
        int si = edge;
        if (g.periodic[axis]) si = ((gi % nd) + nd) % nd;
        F[(long long)(gi + G) * sd] = F[(long long)(si + G) * sd];
    }
}

// ---------------------------------------------------------------------------
// Sigma source and Jacobi sweep
// ---------------------------------------------------------------------------

template <class T, class C>
__device__ __forceinline__ void velocity(const T* U, long long fs, long long o, C u[3]) {
    using S = Storage<T>;
    const C r = C(1) / S::load(U + o);
    u[0] = S::load(U + fs + o) * r;
    u[1] = S::load(U + 2 * fs + o) * r;
    u[2] = S::load(U + 3 * fs + o) * r;
}

// b = alpha [sum_ij G_ij G_ji + (G_xx + G_yy + G_zz)^2], G_ij = d u_i / d x_j
// by central differences (needs one ghost layer of U).
template <class T, class C>
__global__ __launch_bounds__(256) void k_source(const T* __restrict__ U, C* __restrict__ b, Geom g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const long long o = cell_offset(g, i, j, k);
    C Gm[3][3];
    for (int d = 0; d < 3; ++d) {
        C up[3], um[3];
        velocity<T, C>(U, g.fs, o + g.st[d], up);
        velocity<T, C>(U, g.fs, o - g.st[d], um);
        const C s = C(0.5) * C(g.ih[d]);
        for (int c = 0; c < 3; ++c) Gm[c][d] = (up[c] - um[c]) * s;
    }
    const C tr = Gm[0][0] + Gm[1][1] + Gm[2][2];
    C tr2 = C(0);
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) tr2 += Gm[c][d] * Gm[d][c];
    b[o] = C(g.alpha) * (tr2 + tr * tr);
}

// Sigma_out = [b + alpha sum_d (beta+ S+ + beta- S-)/h^2]
//           / [1/rho + alpha sum_d (beta+ + beta-)/h^2],
// beta+- = (1/rho_c + 1/rho_nb)/2; S+- from Sigma_in with periodic wrap or
// zero gradient (Sigma_in ghosts are not read); rho ghosts are read.
template <class T, class C>
__global__ __launch_bounds__(256) void k_jacobi(const T* __restrict__ Sin, T* __restrict__ Sout, const C* __restrict__ b,
                         const T* __restrict__ rho, Geom g) {
    using S = Storage<T>;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const int idx[3] = {i, j, k};
    const long long o = cell_offset(g, i, j, k);
    const C ic = C(1) / S::load(rho + o);
    C num = b[o];
    C den = ic;
    for (int d = 0; d < 3; ++d) {
        const C h2 = C(g.ih[d]) * C(g.ih[d]);
        const C bp = C(0.5) * (ic + C(1) / S::load(rho + o + g.st[d]));
        const C bm = C(0.5) * (ic + C(1) / S::load(rho + o - g.st[d]));
        const C sp = S::load(Sin + o + neighbour_no_ghost(g, d, idx[d], +1));
        const C sm = S::load(Sin + o + neighbour_no_ghost(g, d, idx[d], -1));
        num += C(g.alpha) * (bp * sp + bm * sm) * h2;
        den += C(g.alpha) * (bp + bm) * h2;
    }
    S::store(Sout + o, num / den);
}

// ---------------------------------------------------------------------------
// Reconstruction + local Lax-Friedrichs flux
// ---------------------------------------------------------------------------

// Fifth-order linear reconstruction from cell averages (WENO5 optimal
// weights): left state at face i+1/2 from cells i-2..i+2, right state from
// cells i-1..i+3 (mirror image).  In FP64 the integer-weight sum is scaled
// by the rounded constant 1/60 (a correctly rounded division costs an order
// of magnitude more instructions); in FP32 arithmetic, where the flux
// kernel is bound by instruction issue, the weights are pre-divided (one
// instruction fewer per value: 3 % of the kernel; in FP64 the longer-lived
// constants cost the kernel spills).
template <class C>
__device__ __forceinline__ C recon_left(C a, C b, C c, C d, C e) {
    if constexpr (sizeof(C) == 4)
        return C(2.0 / 60) * a - C(13.0 / 60) * b + C(47.0 / 60) * c + C(27.0 / 60) * d - C(3.0 / 60) * e;
    else
        return (C(2) * a - C(13) * b + C(47) * c + C(27) * d - C(3) * e) * (C(1) / C(60));
}
template <class C>
__device__ __forceinline__ C recon_right(C b, C c, C d, C e, C f) {
    if constexpr (sizeof(C) == 4)
        return C(-3.0 / 60) * b + C(27.0 / 60) * c + C(47.0 / 60) * d - C(13.0 / 60) * e + C(2.0 / 60) * f;
    else
        return (C(-3) * b + C(27) * c + C(47) * d - C(13) * e + C(2) * f) * (C(1) / C(60));
}

// Third-order linear reconstruction (the paper's other order,
// "Discretization"; the optimal linear weights of WENO3): left state at
// face i+1/2 from cells i-1..i+1, right state from cells i..i+2.
template <class C>
__device__ __forceinline__ C recon3_left(C b, C c, C d) {
    return (C(-1) * b + C(5) * c + C(2) * d) * (C(1) / C(6));
}
template <class C>
__device__ __forceinline__ C recon3_right(C c, C d, C e) {
    return (C(2) * c + C(5) * d - C(1) * e) * (C(1) / C(6));
}

// Square root of a sound speed.  FP64: the hardware reciprocal-square-root
// estimate refined by two Goldschmidt steps (g -> sqrt(x), h -> 1/(2 sqrt(x))),
// within about an ulp; the argument gamma p / rho is a positive normal
// number for every state the kernels accept (others are flagged), so the
// range scaling and special-value handling of the library square root are
// left out.  FP32: the hardware instruction (1 ulp).
__device__ __forceinline__ double face_sqrt(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    double h = 0.5 * y;
    const double r = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    double d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    d = __builtin_fma(-g, g, x);
    return __builtin_fma(d, h, g);
}
__device__ __forceinline__ float face_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// LLF (Rusanov) flux along axis d of eqs. (6)-(8) with tau = 0:
// F = 1/2 (F(UL, SL) + F(UR, SR)) - 1/2 lambda (UR - UL),
// lambda = max(|u_n| + c) of the two states (thermodynamic p only).
// Returns F / LLF_SCALE (2F in FP32 arithmetic, F in FP64).
template <class C>
__device__ __forceinline__ void llf_flux(const C UL[5], const C UR[5], C SL, C SR, int d, C gamma,
                                         C F[5], bool& bad) {
    const C irl = fast_rcp(UL[0]);
    const C irr = fast_rcp(UR[0]);
    const C pl = (gamma - C(1)) * (UL[4] - C(0.5) * (UL[1] * UL[1] + UL[2] * UL[2] + UL[3] * UL[3]) * irl);
    const C pr = (gamma - C(1)) * (UR[4] - C(0.5) * (UR[1] * UR[1] + UR[2] * UR[2] + UR[3] * UR[3]) * irr);
    bad |= !(UL[0] > C(0)) | !(UR[0] > C(0)) | !(pl > C(0)) | !(pr > C(0));
    const C unl = UL[1 + d] * irl;
    const C unr = UR[1 + d] * irr;
    const C cl = face_sqrt(gamma * pl * irl);
    const C cr = face_sqrt(gamma * pr * irr);
    const C lam = fmax(fabs(unl) + cl, fabs(unr) + cr);
    const C ptl = pl + SL;
    const C ptr = pr + SR;
    // FP32 arithmetic: twice the flux, one instruction fewer per component
    // (the kernel is issue-bound there; the factor 1/2 goes with the 1/dx
    // of the divergence, LLF_SCALE); FP64 keeps the flux itself (the
    // kernel is at its register limit and the other form spills)
    constexpr C h = sizeof(C) == 4 ? C(1) : C(0.5);
    F[0] = h * (UL[1 + d] + UR[1 + d]) - h * lam * (UR[0] - UL[0]);
    for (int c = 0; c < 3; ++c) {
        C fl = UL[1 + c] * unl;
        C fr = UR[1 + c] * unr;
        if (c == d) {
            fl += ptl;
            fr += ptr;
        }
        F[1 + c] = h * (fl + fr) - h * lam * (UR[1 + c] - UL[1 + c]);
    }
    F[4] = h * ((UL[4] + ptl) * unl + (UR[4] + ptr) * unr) - h * lam * (UR[4] - UL[4]);
}

// Factor between llf_flux's result and the flux: 1/2 in FP32 arithmetic.
template <class C>
constexpr C LLF_SCALE = sizeof(C) == 4 ? C(0.5) : C(1);

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions: fixed grid, grid-stride loop, fixed-order
// block tree; the final pass runs in one block.
// ---------------------------------------------------------------------------

constexpr int RED_THREADS = 256;
constexpr int RED_BLOCKS = 1024;

template <class Op, int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], Op op) {
    __shared__ double sh[NV][RED_THREADS];
    for (int c = 0; c < NV; ++c) sh[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int c = 0; c < NV; ++c) sh[c][threadIdx.x] = op(sh[c][threadIdx.x], sh[c][threadIdx.x + s]);
        __syncthreads();
    }
    for (int c = 0; c < NV; ++c) v[c] = sh[c][0];
}

struct MaxOp {
    __device__ double operator()(double a, double b) const { return fmax(a, b); }
};
struct SumOp {
    __device__ double operator()(double a, double b) const { return a + b; }
};

// CFL speed of one cell, sum_d (|u_d| + c)/h_d, in FP64 whatever the
// storage (the time-step rule of reading R10); flags rho <= 0 or p <= 0.
// Shared by the standalone reduction and the one fused into the last RK
// stage, so both give the same maximum.
__device__ __forceinline__ double cfl_speed(const Geom& g, double rho, double mx, double my, double mz, double E,
                                            bool& bad) {
    const double p = (g.gamma - 1.0) * (E - 0.5 * (mx * mx + my * my + mz * mz) / rho);
    bad |= !(rho > 0.0) | !(p > 0.0);
    const double c = sqrt(g.gamma * p / rho);
    return (fabs(mx / rho) + c) * g.ih[0] + (fabs(my / rho) + c) * g.ih[1] + (fabs(mz / rho) + c) * g.ih[2];
}

// max over cells of sum_d (|u_d| + c)/h_d, in FP64 whatever the storage.
template <class T>
__global__ void k_speed_partial(const T* __restrict__ U, Geom g, double* __restrict__ partial,
                                int* __restrict__ flag) {
    using S = Storage<T>;
    const long long ncell = (long long)g.n[0] * g.n[1] * g.n[2];
    double m[1] = {0.0};
    bool bad = false;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < ncell;
         t += (long long)gridDim.x * blockDim.x) {
        const int i = int(t % g.n[0]);
        const long long r = t / g.n[0];
        const int j = int(r % g.n[1]);
        const int k = int(r / g.n[1]);
        const long long o = cell_offset(g, i, j, k);
        const double s = cfl_speed(g, double(S::load(U + o)), double(S::load(U + g.fs + o)),
                                   double(S::load(U + 2 * g.fs + o)), double(S::load(U + 3 * g.fs + o)),
                                   double(S::load(U + 4 * g.fs + o)), bad);
        m[0] = fmax(m[0], s);
    }
    if (bad) flag[0] = 1;
    block_reduce(m, MaxOp());
    if (threadIdx.x == 0) partial[blockIdx.x] = m[0];
}

// dt = cfl / max(partial); written to *dt_out.
__global__ void k_dt_final(const double* __restrict__ partial, int nblocks, double cfl,
                           double* __restrict__ dt_out) {
    double m[1] = {0.0};
    for (int t = threadIdx.x; t < nblocks; t += blockDim.x) m[0] = fmax(m[0], partial[t]);
    block_reduce(m, MaxOp());
    if (threadIdx.x == 0) dt_out[0] = cfl / m[0];
}

template <class T>
__global__ void k_sums_partial(const T* __restrict__ U, Geom g, double* __restrict__ partial) {
    using S = Storage<T>;
    const long long ncell = (long long)g.n[0] * g.n[1] * g.n[2];
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < ncell;
         t += (long long)gridDim.x * blockDim.x) {
        const int i = int(t % g.n[0]);
        const long long r = t / g.n[0];
        const int j = int(r % g.n[1]);
        const int k = int(r / g.n[1]);
        const long long o = cell_offset(g, i, j, k);
        for (int f = 0; f < 5; ++f) v[f] += double(S::load(U + f * g.fs + o));
    }
    block_reduce(v, SumOp());
    if (threadIdx.x == 0)
        for (int f = 0; f < 5; ++f) partial[f * gridDim.x + blockIdx.x] = v[f];
}

template <int NV>
__global__ void k_sum_final(const double* __restrict__ partial, int nblocks, double scale,
                            double* __restrict__ out) {
    double v[NV];
    for (int c = 0; c < NV; ++c) v[c] = 0.0;
    for (int t = threadIdx.x; t < nblocks; t += blockDim.x)
        for (int c = 0; c < NV; ++c) v[c] += partial[c * nblocks + t];
    block_reduce(v, SumOp());
    if (threadIdx.x == 0)
        for (int c = 0; c < NV; ++c) out[c] = v[c] * scale;
}

// Squared residual of eq. (9)'s discretisation, r = b - A Sigma, in FP64
// (Sigma stored as TS, rho as TR).
template <class TS, class TR, class C>
__global__ void k_resid_partial(const TS* __restrict__ Sg, const C* __restrict__ b, const TR* __restrict__ rho,
                                Geom g, double* __restrict__ partial) {
    using SS = Storage<TS>;
    using SR = Storage<TR>;
    const long long ncell = (long long)g.n[0] * g.n[1] * g.n[2];
    double v[1] = {0.0};
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < ncell;
         t += (long long)gridDim.x * blockDim.x) {
        const int idx[3] = {int(t % g.n[0]), int((t / g.n[0]) % g.n[1]), int(t / g.n[0] / g.n[1])};
        const long long o = cell_offset(g, idx[0], idx[1], idx[2]);
        const double ic = 1.0 / double(SR::load(rho + o));
        const double sc = double(SS::load(Sg + o));
        double a = sc * ic;
        for (int d = 0; d < 3; ++d) {
            const double h2 = g.ih[d] * g.ih[d];
            const double bp = 0.5 * (ic + 1.0 / double(SR::load(rho + o + g.st[d])));
            const double bm = 0.5 * (ic + 1.0 / double(SR::load(rho + o - g.st[d])));
            const double sp = double(SS::load(Sg + o + neighbour_no_ghost(g, d, idx[d], +1)));
            const double sm = double(SS::load(Sg + o + neighbour_no_ghost(g, d, idx[d], -1)));
            a -= g.alpha * (bp * (sp - sc) - bm * (sc - sm)) * h2;
        }
        const double r = double(b[o]) - a;
        v[0] += r * r;
    }
    block_reduce(v, SumOp());
    if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

}  // namespace igr
