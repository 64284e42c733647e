// Temporally blocked Sigma solve: source + K Jacobi sweeps in one pass.
//
// A block owns an extended tile of 64 x NR columns (the output tile plus a
// K-cell halo on each side in x and y) and marches through a chunk of z
// planes as a wavefront: when input plane P (rho, m) arrives, the source b
// is formed at plane P-1 and Jacobi level s (1..K) updates plane P-1-s,
// so level K emits output plane P-1-K.  Each column keeps the z
// neighbours of every level in registers; the x/y neighbours of the plane a
// level reads were written to LDS in the previous iteration (one slot per
// level, a K-slot ring for 1/rho, one slot for u).  Two barriers per plane:
// phase R reads LDS and computes, phase W publishes the new planes.
//
// Boundaries: periodic axes wrap the input indices, so halo columns and
// planes compute exactly the wrapped values; on zero-gradient axes the
// missing Sigma neighbour of a boundary cell is the cell itself (the ghost
// equals the previous iterate of the first interior cell) while rho and u
// use the filled ghost layer of U, as in the one-sweep kernel.
#pragma once

#include "igr_kernels.h"

namespace igr {

constexpr int SIG_TX = 64;

// One Jacobi update of the 7-point discretisation of eq. (9) at a cell,
// in two parts: the coefficients (the face sums 1/rho_c + 1/rho_nb = 2 beta
// and the reciprocal of the diagonal) depend on 1/rho only and are shared
// by every sweep of a solve; the update combines them with the source and
// the previous iterate, the factor 1/2 of beta carried with alpha/h^2 in
// one constant per axis (loop-invariant in the callers).  ic = 1/rho of
// the cell, ir = 1/rho and sg = the previous iterate at the x-, x+, y-,
// y+, z-, z+ neighbours (sg already replaced by the cell's own value where
// a zero-gradient face removes the neighbour).  Every sweep kernel goes
// through these two functions, so equal inputs give equal bits.
template <class C>
struct JacCoef {
    C bxm, bxp, bym, byp, bzm, bzp;   // 2 beta of the six faces
    C rden;                           // 1 / (1/rho + alpha sum_d (beta_d- + beta_d+)/h_d^2)
};

// alpha / (2 h_d^2) per axis: the constants the update needs, from the
// geometry (every kernel forms them the same way)
template <class C>
struct JacAxes {
    C ax, ay, az;
};
template <class C>
__device__ __forceinline__ JacAxes<C> jacobi_axes(const Geom& g) {
    const C ha = C(0.5) * C(g.alpha);
    return {ha * (C(g.ih[0]) * C(g.ih[0])), ha * (C(g.ih[1]) * C(g.ih[1])), ha * (C(g.ih[2]) * C(g.ih[2]))};
}

template <class C>
__device__ __forceinline__ JacCoef<C> jacobi_coef(C ic, const C (&ir)[6], const JacAxes<C>& a) {
    JacCoef<C> k;
    k.bxm = ic + ir[0];
    k.bxp = ic + ir[1];
    k.bym = ic + ir[2];
    k.byp = ic + ir[3];
    k.bzm = ic + ir[4];
    k.bzp = ic + ir[5];
    C den = ic;
    den += a.ax * (k.bxp + k.bxm);
    den += a.ay * (k.byp + k.bym);
    den += a.az * (k.bzp + k.bzm);
    k.rden = fast_rcp(den);
    return k;
}

template <class C>
__device__ __forceinline__ C jacobi_apply(C bk, const JacCoef<C>& k, const C (&sg)[6], const JacAxes<C>& a) {
    C num = bk;
    num += a.ax * (k.bxp * sg[1] + k.bxm * sg[0]);
    num += a.ay * (k.byp * sg[3] + k.bym * sg[2]);
    num += a.az * (k.bzp * sg[5] + k.bzm * sg[4]);
    return num * k.rden;
}

template <class C>
__device__ __forceinline__ C jacobi_point(C bk, C ic, const C (&ir)[6], const C (&sg)[6], const JacAxes<C>& a) {
    return jacobi_apply(bk, jacobi_coef(ic, ir, a), sg, a);
}


template <class T, int K, int NR>
__global__ __launch_bounds__(SIG_TX* NR) void k_sigma_march(const T* __restrict__ U, const T* __restrict__ Sin,
                                                           T* __restrict__ Sout, Geom g, int tiles_x, int tiles_y,
                                                           int zc) {
    using S = Storage<T>;
    using C = typename S::C;
    constexpr int TXo = SIG_TX - 2 * K;
    constexpr int TYo = NR - 2 * K;
    static_assert(TYo >= 1, "tile too small for K levels");
    __shared__ C lu[3][NR][SIG_TX];        // u at plane P-1
    __shared__ C ls[K][NR][SIG_TX];        // level l at plane P-2-l (for level l+1)
    __shared__ C lr[K][NR][SIG_TX];        // 1/rho ring, slot = plane mod K

    const int ex = threadIdx.x;
    const int ey = threadIdx.y;
    int bidx = blockIdx.x;
    {
        constexpr int NXCD = 8;
        const int nb = gridDim.x;
        const int full = nb - nb % NXCD;
        if (bidx < full) bidx = (bidx % NXCD) * (full / NXCD) + bidx / NXCD;
    }
    const int tx = bidx % tiles_x;
    bidx /= tiles_x;
    const int ty = bidx % tiles_y;
    const int cz = bidx / tiles_y;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int gx = tx * TXo - K + ex;    // global column of this thread
    const int gy = ty * TYo - K + ey;
    const int z0 = cz * zc;
    const int z1 = min(z0 + zc, nz);
    const long long fs = g.fs;
    const int sy = g.st[1], sz = g.st[2];
    const C alpha = C(g.alpha);
    const JacAxes<C> ja = jacobi_axes<C>(g);
    const C sx = C(0.5) * C(g.ih[0]), sy_ = C(0.5) * C(g.ih[1]), sz_ = C(0.5) * C(g.ih[2]);

    // source column in memory: periodic axes wrap, other axes clamp to the
    // padded range (only the first ghost layer is ever used there)
    auto src_index = [](int c, int n, int periodic) {
        if (periodic) return ((c % n) + n) % n;
        return c < -G ? -G : (c > n + G - 1 ? n + G - 1 : c);
    };
    const int cx = src_index(gx, nx, g.periodic[0]);
    const int cy = src_index(gy, ny, g.periodic[1]);
    const long long col = (long long)(cy + G) * sy + (cx + G);
    // zero-gradient boundary flags of this column (Sigma neighbour = self)
    const bool xlo = !g.periodic[0] && gx == 0, xhi = !g.periodic[0] && gx == nx - 1;
    const bool ylo = !g.periodic[1] && gy == 0, yhi = !g.periodic[1] && gy == ny - 1;
    const bool out_col = ex >= K && ex < SIG_TX - K && ey >= K && ey < NR - K && gx < nx && gy < ny;
    const int exm = ex > 0 ? ex - 1 : ex, exp_ = ex < SIG_TX - 1 ? ex + 1 : ex;
    const int eym = ey > 0 ? ey - 1 : ey, eyp = ey < NR - 1 ? ey + 1 : ey;

    C uR[3][3];        // u at planes P-2, P-1, P
    C irR[K + 3];      // 1/rho at planes P-d, d = 0..K+2
    C bR[K + 1];       // b at planes P-1-d, d = 0..K
    C lo[K], mid[K];   // level l at planes P-3-l, P-2-l
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int p = 0; p < 3; ++p) uR[c][p] = C(0);
#pragma unroll
    for (int d = 0; d < K + 3; ++d) irR[d] = C(1);
#pragma unroll
    for (int d = 0; d < K + 1; ++d) bR[d] = C(0);
#pragma unroll
    for (int l = 0; l < K; ++l) lo[l] = mid[l] = C(0);

    // LDS starts defined (planes read before the wavefront fills them feed
    // only cells that never reach an output)
    for (int t = ey * SIG_TX + ex; t < NR * SIG_TX; t += NR * SIG_TX) {
        const int r = t / SIG_TX, c = t % SIG_TX;
#pragma unroll
        for (int q = 0; q < 3; ++q) lu[q][r][c] = C(0);
#pragma unroll
        for (int q = 0; q < K; ++q) {
            ls[q][r][c] = C(0);
            lr[q][r][c] = C(1);
        }
    }
    __syncthreads();
    const int pbeg = z0 - K;
    const int pend = z1 + K + 1;   // input planes pbeg .. pend-1 emit outputs z0 .. z1-1
    // inputs of plane P are loaded one iteration ahead (registers nr, nm*, ns)
    auto load_inputs = [&](int P, C& r, C& a, C& b, C& c, C& sg) {
        const int pz = src_index(P, nz, g.periodic[2]);
        const int pzs = src_index(P - 1, nz, g.periodic[2]);
        const long long o = col + (long long)(pz + G) * sz;
        r = S::load(U + o);
        a = S::load(U + fs + o);
        b = S::load(U + 2 * fs + o);
        c = S::load(U + 3 * fs + o);
        sg = S::load(Sin + col + (long long)(pzs + G) * sz);
    };
    C nr, nm0, nm1, nm2, ns;
    load_inputs(pbeg, nr, nm0, nm1, nm2, ns);
    for (int P = pbeg; P < pend; ++P) {
        // ---- inputs: rho, m at plane P; Sigma_0 at plane P-1 (prefetched)
        const C rho = nr;
        const C ir = C(1) / rho;
        const C u0 = nm0 * ir;
        const C u1 = nm1 * ir;
        const C u2 = nm2 * ir;
        const C s0new = ns;
        if (P + 1 < pend) load_inputs(P + 1, nr, nm0, nm1, nm2, ns);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            uR[c][0] = uR[c][1];
            uR[c][1] = uR[c][2];
        }
        uR[0][2] = u0;
        uR[1][2] = u1;
        uR[2][2] = u2;
#pragma unroll
        for (int d = K + 2; d > 0; --d) irR[d] = irR[d - 1];
        irR[0] = ir;

        // ---- phase R: source at plane P-1, level s at plane P-1-s
        C bnew;
        {
            C Gm[3][3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Gm[c][0] = (lu[c][ey][exp_] - lu[c][ey][exm]) * sx;
                Gm[c][1] = (lu[c][eyp][ex] - lu[c][eym][ex]) * sy_;
                Gm[c][2] = (uR[c][2] - uR[c][0]) * sz_;
            }
            const C tr = Gm[0][0] + Gm[1][1] + Gm[2][2];
            C tr2 = C(0);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) tr2 += Gm[c][d] * Gm[d][c];
            bnew = alpha * (tr2 + tr * tr);
        }
        C newv[K + 1];
        newv[0] = s0new;   // level 0 at plane P-1
#pragma unroll
        for (int s = 1; s <= K; ++s) {
            const int zs = P - 1 - s;    // plane updated by level s
            const int zsp = src_index(zs, nz, g.periodic[2]);
            const bool zlo = !g.periodic[2] && zsp == 0 && zs == 0;
            const bool zhi = !g.periodic[2] && zs == nz - 1;
            const int slot = ((zs % K) + K) % K;
            const C ic = irR[1 + s];
            const C sc = mid[s - 1];
            // x/y neighbours of level s-1 and of 1/rho at plane zs
            const C sxm = xlo ? sc : ls[s - 1][ey][exm];
            const C sxp = xhi ? sc : ls[s - 1][ey][exp_];
            const C sym = ylo ? sc : ls[s - 1][eym][ex];
            const C syp = yhi ? sc : ls[s - 1][eyp][ex];
            const C szm = zlo ? sc : lo[s - 1];
            const C szp = zhi ? sc : newv[s - 1];
            const C irv[6] = {lr[slot][ey][exm], lr[slot][ey][exp_], lr[slot][eym][ex],
                              lr[slot][eyp][ex], irR[2 + s],         irR[s]};
            const C sgv[6] = {sxm, sxp, sym, syp, szm, szp};
            // b at plane P-1-s (bR is shifted at the end of the iteration)
            newv[s] = jacobi_point(bR[s - 1], ic, irv, sgv, ja);
        }
        __syncthreads();
        // ---- phase W: publish planes for the next iteration
        lu[0][ey][ex] = u0;
        lu[1][ey][ex] = u1;
        lu[2][ey][ex] = u2;
        {
            const int slot = (((P - 1) % K) + K) % K;   // 1/rho at plane P-1
            lr[slot][ey][ex] = irR[1];
        }
#pragma unroll
        for (int l = 0; l < K; ++l) ls[l][ey][ex] = newv[l];
        {
            const int zo = P - 1 - K;
            if (out_col && zo >= z0 && zo < z1)
                S::store(Sout + (long long)(zo + G) * sz + (long long)(gy + G) * sy + (gx + G), newv[K]);
        }
        // register shifts
#pragma unroll
        for (int d = K; d > 0; --d) bR[d] = bR[d - 1];
        bR[0] = bnew;
#pragma unroll
        for (int l = 0; l < K; ++l) {
            lo[l] = mid[l];
            mid[l] = newv[l];
        }
        __syncthreads();
    }
}

// One Jacobi sweep per pass, z-marching: a 64 x SWEEP_RY block of columns walks a
// chunk of z planes, keeping the z neighbours of Sigma and 1/rho in
// registers; x/y neighbours are read from memory (L1/L2 hits: adjacent
// lanes and rows).  Loads are issued ahead of use (see SweepCol) so that
// enough bytes are in flight per CU to cover HBM latency.  With FIRST the
// source b is formed in the same pass (from rho and m) and written for the
// later sweeps.  Per cell: FIRST reads rho, m, Sigma and writes Sigma, b;
// later sweeps read Sigma, rho, b and write Sigma.  With colour >= 0 the
// kernel runs one half of a red-black Gauss-Seidel sweep in place.
// Loads of one iteration of the single-sweep kernel.  The own-column values
// of plane k+1 (which miss to HBM) are fetched PD iterations ahead; the x/y
// neighbours of plane k (mostly L1/L2 hits: other threads' columns) one
// iteration ahead.
// Values are kept in the storage's register form R (converted where used)
// so that a conversion does not wait for its load.  In FP64 later sweeps
// `rho` holds the stored 1/rho.
// In the later sweeps of a form that stores 1/rho (IRS), `rho` holds the
// stored 1/rho (arithmetic type) instead of a loaded state value.
template <class F, bool FIRST>
struct SweepCol {
    using C = typename F::C;
    using RU = typename F::RU;
    using RR = std::conditional_t<F::IRS && !FIRST, C, RU>;
    RR rho;             // rho (or 1/rho) at plane k+1
    RU sig;             // Sigma_in at plane k+1
    C b;                // b at plane k (later sweeps)
    RU m[3];            // m at plane k+1 (FIRST)
    RU E;               // E at plane k+1 (first sweep that also forms the CFL maxima)
};
template <class F, bool FIRST>
struct SweepNb {
    using RU = typename F::RU;
    using RR = std::conditional_t<F::IRS && !FIRST, typename F::C, RU>;
    RR rho[4];
    RU sig[4];   // x/y neighbours of plane k
    RU m[4][3];  // (FIRST)
};

#ifndef IGR_SWEEP_RY
#define IGR_SWEEP_RY 4
#endif
#ifndef IGR_SWEEP_RY_FIRST
#define IGR_SWEEP_RY_FIRST 4
#endif
constexpr int SWEEP_RY = IGR_SWEEP_RY;               // rows of a later-sweep block (64 x SWEEP_RY)
constexpr int SWEEP_RY_FIRST = IGR_SWEEP_RY_FIRST;   // rows of a first-sweep block

// With SPD (first sweep only) the kernel also reads E and forms the CFL
// speed of every cell of its chunk of the state it sweeps from (cfl_speed,
// the expression of the standalone reduction, on the stored values); each
// wave leaves its maximum in speed[blockIdx.x * RY + wave] and non-physical
// states raise *flag, so the time step of the stage needs no separate pass.
// F: storage form; the state swept from is U (+ D with HASD, the split
// form's stage difference).  TAU (FIRST): the sweep also stores the
// viscous stress of eq. (5) formed from the source's velocity gradients
// (six components, tau_index order) at every cell it stores b at.
template <class F, bool FIRST, int RY, bool SPD = false, bool HASD = false, bool TAU = false>
__global__ __launch_bounds__(64 * RY) void k_sweep_z(const typename F::TB* __restrict__ U,
                                                 const typename F::TD* __restrict__ D, const typename F::TS* Sin,
                                                 typename F::TS* Sout, typename F::C* __restrict__ b,
                                                 typename F::C* __restrict__ irs, Geom g, int zc,
                                                 int tiles_x, int tiles_y, int colour,
                                                 double* __restrict__ speed, int* __restrict__ flag,
                                                 typename F::C* __restrict__ tau = nullptr, double mu_ = 0.0,
                                                 double zeta_ = 0.0) {
    static_assert(!SPD || FIRST, "the CFL maxima need the first sweep's state loads");
    static_assert(!TAU || FIRST, "the stress needs the first sweep's velocity gradients");
    using C = typename F::C;
    using SS = Storage<typename F::TS>;
    constexpr int PD = 3;   // own-column prefetch distance (planes)
    // the split form's first sweep stores 1/rho (interior and the face-ghost
    // layer) and later sweeps read it (one FP32 value instead of a base and
    // a difference)
    constexpr bool IRS = F::IRS;
    // 1-D grid in XCD-aware order: consecutive logical tiles (x fastest,
    // then y, then z chunk) run on one XCD, so rows shared by y-neighbour
    // tiles are fetched once into that XCD's L2
    int bx, by, bz;
    tile_coords(xcd_remap(blockIdx.x, gridDim.x), tiles_x, tiles_y, bx, by, bz);
    const int i = bx * 64 + threadIdx.x;
    const int j = by * RY + threadIdx.y;
    const int z0 = bz * zc;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    double smax = 0.0;   // SPD: CFL maximum of this thread's cells
    bool bad = false;
    // lanes outside the grid skip the sweep (no early return: with SPD every
    // lane takes part in the wave's reduction at the end)
    if (i < nx && j < ny) {
    const int z1 = min(z0 + zc, nz);
    const long long fs = g.fs;
    const int sy = g.st[1], sz = g.st[2];
    const long long col = (long long)(j + G) * sy + (i + G);
    const C alpha = C(g.alpha);
    const JacAxes<C> ja = jacobi_axes<C>(g);
    // x/y neighbours: rho from the padded array, Sigma with wrap or self
    const int onb[4] = {-1, 1, -sy, sy};
    const int osg[4] = {neighbour_no_ghost(g, 0, i, -1), neighbour_no_ghost(g, 0, i, +1),
                        neighbour_no_ghost(g, 1, j, -1), neighbour_no_ghost(g, 1, j, +1)};
    auto zplane = [&](int k) { return col + (long long)(k + G) * sz; };
    auto zsig = [&](int k) {   // Sigma plane of z neighbour k: wrap or self at the ends
        if (k < 0) return g.periodic[2] ? nz - 1 : 0;
        if (k >= nz) return g.periodic[2] ? 0 : nz - 1;
        return k;
    };
    auto ldu = [&](long long o) { return F::template load_u<HASD>(U, D, o); };
    auto getu = [&](long long o) { return F::cvt(ldu(o)); };
    auto load_col = [&](int k, SweepCol<F, FIRST>& P) {   // for iteration k
        const long long op = zplane(k + 1);
        if constexpr (IRS && !FIRST)
            P.rho = irs[op];
        else
            P.rho = ldu(op);
        P.sig = F::load_s(Sin, col + (long long)(zsig(k + 1) + G) * sz);
        if constexpr (FIRST) {
#pragma unroll
            for (int c = 0; c < 3; ++c) P.m[c] = ldu((1 + c) * fs + op);
        } else {
            P.b = b[zplane(k)];
        }
        if constexpr (SPD) P.E = ldu(4 * fs + op);
    };
    auto load_nb = [&](int k, SweepNb<F, FIRST>& P) {
        const long long o = zplane(k);
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            if constexpr (IRS && !FIRST)
                P.rho[n] = irs[o + onb[n]];
            else
                P.rho[n] = ldu(o + onb[n]);
            P.sig[n] = F::load_s(Sin, o + osg[n]);
        }
        if constexpr (FIRST) {
#pragma unroll
            for (int n = 0; n < 4; ++n)
#pragma unroll
                for (int c = 0; c < 3; ++c) P.m[n][c] = ldu((1 + c) * fs + o + onb[n]);
        }
    };
    // v: rho (register form), or 1/rho stored (later sweeps of an IRS form)
    auto inv_rho = [&](auto v) -> C {
        if constexpr (IRS && !FIRST)
            return v;
        else
            return fast_rcp(F::cvt(v));
    };
    C ir_m, ir_c;
    if constexpr (IRS && !FIRST) {
        ir_m = irs[zplane(z0 - 1)];
        ir_c = irs[zplane(z0)];
    } else {
        ir_m = fast_rcp(getu(zplane(z0 - 1)));
        ir_c = fast_rcp(getu(zplane(z0)));
    }
    C s_m = F::cvt(F::load_s(Sin, col + (long long)(zsig(z0 - 1) + G) * sz));
    C s_c = F::cvt(F::load_s(Sin, zplane(z0)));
    C u_m[3], u_c[3];
    if constexpr (FIRST) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            u_m[c] = getu((1 + c) * fs + zplane(z0 - 1)) * ir_m;
            u_c[c] = getu((1 + c) * fs + zplane(z0)) * ir_c;
        }
    }
    if constexpr (SPD) {   // plane z0; the loop adds plane k+1 < z1 at iteration k
        const long long o0 = zplane(z0);
        smax = cfl_speed(g, double(getu(o0)), double(getu(fs + o0)), double(getu(2 * fs + o0)),
                         double(getu(3 * fs + o0)), double(getu(4 * fs + o0)), bad);
    }
    // Loads are unconditional (planes clamped to the chunk) and issued in
    // the order they are needed -- the neighbours of the next plane first,
    // then the own column PD planes ahead -- because vector-memory counters
    // complete in order: waiting for the neighbours must not wait for the
    // look-ahead.  The loop is unrolled over the register rotation so that
    // the rotation is renaming, not copies of pending loads.
    SweepCol<F, FIRST> q[PD];   // own columns for iterations k .. k+PD-1
#pragma unroll
    for (int d = 0; d < PD; ++d) load_col(min(z0 + d, z1 - 1), q[d]);
    SweepNb<F, FIRST> cur, nxt;
    load_nb(z0, cur);
#pragma unroll 6
    for (int k = z0; k < z1; ++k) {
        const SweepCol<F, FIRST> cc = q[0];
#pragma unroll
        for (int d = 0; d < PD - 1; ++d) q[d] = q[d + 1];
        load_nb(min(k + 1, z1 - 1), nxt);
        load_col(min(k + PD, z1 - 1), q[PD - 1]);
        const long long o = zplane(k);
        const C ir_p = inv_rho(cc.rho);
        const C s_p = F::cvt(cc.sig);
        C irn[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) irn[n] = inv_rho(cur.rho[n]);
        if (IRS && FIRST) {
            irs[o] = ir_c;
            if (i == 0) irs[o - 1] = irn[0];
            if (i == nx - 1) irs[o + 1] = irn[1];
            if (j == 0) irs[o - sy] = irn[2];
            if (j == ny - 1) irs[o + sy] = irn[3];
            if (k == 0) irs[o - sz] = ir_m;
            if (k == nz - 1) irs[o + sz] = ir_p;
        }
        C bk;
        C u_p[3];
        if (FIRST) {
#pragma unroll
            for (int c = 0; c < 3; ++c) u_p[c] = F::cvt(cc.m[c]) * ir_p;
            C Gm[3][3];
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                const C sc = C(0.5) * C(g.ih[d]);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    Gm[c][d] = (F::cvt(cur.m[2 * d + 1][c]) * irn[2 * d + 1] - F::cvt(cur.m[2 * d][c]) * irn[2 * d]) * sc;
            }
            const C scz = C(0.5) * C(g.ih[2]);
#pragma unroll
            for (int c = 0; c < 3; ++c) Gm[c][2] = (u_p[c] - u_m[c]) * scz;
            const C tr = Gm[0][0] + Gm[1][1] + Gm[2][2];
            C tr2 = C(0);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) tr2 += Gm[c][d] * Gm[d][c];
            bk = alpha * (tr2 + tr * tr);
            b[o] = bk;
            if constexpr (TAU) {
                const C mu = C(mu_), lam = C(zeta_) - C(2) * C(mu_) / C(3);
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int e = a; e < 3; ++e) {
                        C t = mu * (Gm[a][e] + Gm[e][a]);
                        if (a == e) t += lam * tr;
                        tau[(long long)tau_index(a, e) * g.fs + o] = t;
                    }
            }
        } else {
            bk = cc.b;
        }
        const C irv[6] = {irn[0], irn[1], irn[2], irn[3], ir_m, ir_p};
        const C sgv[6] = {F::cvt(cur.sig[0]), F::cvt(cur.sig[1]), F::cvt(cur.sig[2]), F::cvt(cur.sig[3]), s_m, s_p};
        // colour < 0: every cell (Jacobi, Sout != Sin); else only the cells
        // with (i + j + k) % 2 == colour, in place (red-black Gauss-Seidel:
        // with even periodic extents every neighbour read here has the
        // other colour, so no value this launch writes is read by it)
        if (colour < 0 || ((i + j + k) & 1) == colour)
            SS::store(Sout + o, jacobi_point(bk, ir_c, irv, sgv, ja));
        if constexpr (SPD) {
            if (k + 1 < z1)
                smax = fmax(smax, cfl_speed(g, double(F::cvt(cc.rho)), double(F::cvt(cc.m[0])),
                                            double(F::cvt(cc.m[1])), double(F::cvt(cc.m[2])),
                                            double(F::cvt(cc.E)), bad));
        }
        ir_m = ir_c;
        ir_c = ir_p;
        s_m = s_c;
        s_c = s_p;
        if (FIRST) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                u_m[c] = u_c[c];
                u_c[c] = u_p[c];
            }
        }
        cur = nxt;
    }
    }
    if constexpr (SPD) {
        for (int off = 32; off > 0; off >>= 1) smax = fmax(smax, __shfl_xor(smax, off, 64));
        if (threadIdx.x == 0) speed[(long long)blockIdx.x * RY + threadIdx.y] = smax;
        if (bad) flag[0] = 1;
    }
}


// Two Jacobi sweeps per pass over memory, for the sweeps after the first
// one of a solve (the source b and, in the split form, 1/rho were stored by the
// first sweep).  A block of 64 x NR threads owns the columns x0..x0+63 of
// rows y0-1..y0+NR-2 and marches through a chunk of z planes; its output
// is the 64 x (NR-2) tile of rows y0..y0+NR-3 (level 2 needs level 1 on a
// one-cell ring around it, level 1 needs the input on a two-cell ring).
// One more wave holds the columns beside the tile: x0-1 and x0+64 (level 1
// is formed there too) and x0-2 and x0+65 (input only); every row wave
// also loads the row y0-2 (row 0) or y0+NR-1 (row NR-1) -- the other rows
// load their own column a second time, so that every lane issues the same
// loads.
//
// z-wavefront: in iteration P the input plane P (Sigma, 1/rho, b) arrives
// and is written to LDS rings, level 1 is formed at plane P-1 and level 2
// (the output) at plane P-2.  Every input, the z neighbours included, is
// read back from the rings; only level 1 (and the coefficients and source
// of the cell level 1 formed last, which level 2 reuses one plane later)
// is kept in registers.  The rings are sized so that one barrier per plane
// suffices: while a wave still reads planes P, P-1, P-2 another may
// already publish plane P+1 (Sigma and 1/rho: 4 slots, b: 3, level 1: 2).
// Loads run PD = 2 planes ahead in two register slots; the plane loop is
// unrolled by two so that each slot is refilled by its own instructions,
// and a slot's only consumer is the LDS write: vector-memory counters
// complete in order, so a register copy of a pending load, or a load under
// a branch, would make every iteration wait for all loads in flight.
// Indices outside the grid wrap on periodic axes and clamp elsewhere;
// cells whose value is then not the true one (beyond a zero-gradient
// face) only feed cells beyond that face, never an output: at a
// zero-gradient face the missing Sigma neighbour is the cell itself.
// The intermediate level stays in the arithmetic type (it is never stored).
#ifndef IGR_PAIR_NR
#define IGR_PAIR_NR 11
#endif
constexpr int PAIR_NR = IGR_PAIR_NR;   // rows per pair block (output NR-2), FP32 arithmetic
// Rows per block, measured at 1024^3: FP64 later passes 15 (16 waves, one
// block per CU: 117 VGPRs, 111 KB of LDS; (15 + 2) / 13 input rows per
// output row instead of (7 + 2) / 5); FP32-arithmetic later passes 11 (two
// blocks of 12 waves per CU; 13 and 15 rows were slower)
#ifndef IGR_PAIR_NR_F64
#define IGR_PAIR_NR_F64 15
#endif
template <class F>
constexpr int pair_nr_later() {
    return std::is_same_v<typename F::C, double> ? IGR_PAIR_NR_F64 : PAIR_NR;
}

#ifndef IGR_PAIR_NR_FIRST
#define IGR_PAIR_NR_FIRST 7
#endif
constexpr int PAIR_NR_FIRST = IGR_PAIR_NR_FIRST;   // rows per block of the first pass of a solve
// First pass (without the CFL maxima): rows per block by arithmetic type,
// measured at 1024^3: FP64 11 (12 waves at 168 VGPRs, 132 KB of LDS:
// 21.4 -> 17.0 ms per launch against 7 rows; 13 rows spill), FP32 15
// (9.2 -> 7.9 ms), the split form's first pass of a later stage 15 (13.3 ->
// 12.2 ms).  The FP64 first pass that also forms the CFL maxima keeps
// PAIR_NR_FIRST (213 VGPRs at 2 waves per SIMD).
#ifndef IGR_PAIR_NR_FIRST_F64
#define IGR_PAIR_NR_FIRST_F64 11
#endif
#ifndef IGR_PAIR_NR_FIRST_F32
#define IGR_PAIR_NR_FIRST_F32 15
#endif
#ifndef IGR_PAIR_NR_FIRST_HASD
#define IGR_PAIR_NR_FIRST_HASD 15
#endif
template <class F, bool HASD>
constexpr int pair_nr_first() {
    return std::is_same_v<typename F::C, double> ? IGR_PAIR_NR_FIRST_F64
                                                 : (HASD ? IGR_PAIR_NR_FIRST_HASD : IGR_PAIR_NR_FIRST_F32);
}

// Sigma neighbour of a cell: the LDS value, or the cell's own value `sc`
// across a zero-gradient face.  With SEL the read is unconditional and the
// choice a select; otherwise a branch skips the read.  (The LDS value comes
// by pointer: through a reference the compiler would speculate the read
// either way.)
template <bool SEL, class C>
__device__ __forceinline__ C face_or(bool face, C sc, const C* nb) {
    if constexpr (SEL) {
        const C t = *nb;
        return face ? sc : t;
    } else {
        return face ? sc : *nb;
    }
}

template <class F, bool FIRST>
struct PairIn;
template <class F>
struct PairIn<F, false> {   // loads of one plane for one thread (register form RU)
    using C = typename F::C;
    using RU = typename F::RU;
    using RR = std::conditional_t<F::IRS, C, RU>;   // rho, or the stored 1/rho
    RU s0;          // own column: Sigma
    RR ir;          // own column: rho (or 1/rho when stored)
    C b;            // own column: b
    RU xs0;         // the ring-2 row (rows 0 and NR-1; others: own column)
    RR xir;
};
template <class F>
struct PairIn<F, true> {    // first pass of a solve: the state instead of b and 1/rho
    using RU = typename F::RU;
    RU s0, rho, m[3];
    RU xs0, xrho, xm[3];
    RU E;                   // own column (a first pass that also forms the CFL maxima)
};

// FIRST: the first pass of a solve, which also forms the source b (eq. 9's
// left side, second-order central velocity gradients) at every level-1
// cell from u = m/rho in LDS (x/y neighbours) and a register queue (z), and
// stores b and, in the split form, 1/rho for the later passes -- the work of the
// single first sweep fused into the pair.  With SPD (FIRST) it also loads
// E and forms the CFL speed (cfl_speed, the standalone reduction's
// expression) of every interior cell of its output tile and chunk; each
// wave leaves its maximum in speed[blockIdx.x * (NR + 1) + wave] and
// non-physical states raise *flag.
// F: storage form; the state swept from is U (+ D with HASD, the split
// form's stage difference).
// TAU (FIRST): the pass also stores the viscous stress of eq. (5) formed
// from the same velocity gradients, tau_ab = mu (G_ab + G_ba) +
// (zeta - 2 mu / 3) tr(G) delta_ab, at the cells where it stores b (six
// components, tau_index order; interior cells).
// RB: one red-black Gauss-Seidel sweep instead of two Jacobi sweeps:
// level 1 applies the update to the red cells ((i + j + k) even) and keeps
// the black ones, level 2 applies it to the black cells from level 1's
// values and keeps the red ones.  Every neighbour of a cell has the other
// colour, so level 1 is the red half-sweep from the values at its start
// and level 2 the black half-sweep (a zero-gradient face reads the cell's
// own value at the start of its half: the old value for red, level 1's
// for black); periodic axes must have even extents.
#ifndef IGR_SPLIT_FIRST_MINW
#define IGR_SPLIT_FIRST_MINW 4
#endif
template <class F, int NR, bool FIRST, bool HASD = false, bool SPD = false, bool RB = false, bool TAU = false>
__global__ __launch_bounds__(64 * (NR + 1), (F::SPLIT && FIRST && HASD) ? IGR_SPLIT_FIRST_MINW : 1) void k_sweep_pair(const typename F::TB* __restrict__ U,
                                                            const typename F::TD* __restrict__ D,
                                                            const typename F::TS* __restrict__ Sin,
                                                            typename F::TS* __restrict__ Sout,
                                                            typename F::C* __restrict__ b,
                                                            typename F::C* __restrict__ irs, Geom g,
                                                            int zc, int tiles_x, int tiles_y,
                                                            double* __restrict__ speed = nullptr,
                                                            int* __restrict__ flag = nullptr,
                                                            typename F::C* __restrict__ tau = nullptr,
                                                            double mu_ = 0.0, double zeta_ = 0.0) {
    static_assert(!SPD || FIRST, "the CFL maxima need the first pass's state loads");
    static_assert(!TAU || FIRST, "the stress needs the first pass's velocity gradients");
    using C = typename F::C;
    using SS = Storage<typename F::TS>;
    constexpr bool IRS = F::IRS;           // 1/rho stored by the first pass (split form)
    constexpr int PD = 2;                   // planes loaded ahead (= register slots)
    constexpr int W0 = 68;                  // input row: columns x0-2 .. x0+65
    constexpr int W1 = 66;                  // level-1 and b row: x0-1 .. x0+64
    __shared__ C ls0[4][NR + 2][W0];
    __shared__ C lir[4][NR + 2][W0];
    __shared__ C lb[FIRST ? 1 : 3][FIRST ? 1 : NR][FIRST ? 1 : W1];
    __shared__ C lu[FIRST ? 3 : 1][FIRST ? 3 : 1][FIRST ? NR + 2 : 1][FIRST ? W0 : 1];
    __shared__ C ls1[2][NR][W1];
    static_assert(4 * NR - 4 <= 64, "side columns must fit one wave");
#ifndef IGR_PAIR_NBSEL
#define IGR_PAIR_NBSEL 1
#endif
    // neighbour reads as selects in the FP32-arithmetic kernels (not in the
    // split form's first pass of a later stage, where they would cost it a
    // wave per SIMD: 129 VGPRs)
    constexpr bool NBSEL = IGR_PAIR_NBSEL && sizeof(C) == 4 && !(FIRST && HASD && IGR_SPLIT_FIRST_MINW < 4);

    int bx, by, bz;
    tile_coords(xcd_remap(blockIdx.x, gridDim.x), tiles_x, tiles_y, bx, by, bz);
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int x0 = bx * 64, y0 = by * (NR - 2), z0 = bz * zc;
    const int z1 = min(z0 + zc, nz);
    const int px = g.periodic[0], py = g.periodic[1], pz = g.periodic[2];
    const long long fs = g.fs;

    // role of this thread: its column (lx, ly) in tile coordinates
    int lx = threadIdx.x, ly = threadIdx.y;
    bool act = true, lev1 = true, hasb = true;
    if (threadIdx.y == NR) {
        const int h = threadIdx.x;
        if (h < 2 * NR) {                       // x0-1 / x0+64, every row
            lx = h < NR ? -1 : 64;
            ly = h % NR;
            lev1 = ly >= 1 && ly <= NR - 2;
        } else if (h < 4 * NR - 4) {            // x0-2 / x0+65, rows 1..NR-2
            const int q = h - 2 * NR;
            lx = q < NR - 2 ? -2 : 65;
            ly = 1 + q % (NR - 2);
            lev1 = false;
            hasb = false;
        } else {                                // spare lanes: load x0-2 of row 1, publish nothing
            act = false;
            lev1 = false;
            hasb = false;
            lx = -2;
            ly = 1;
        }
    }
    const int gx = x0 + lx, gy = y0 - 1 + ly;
    const int par = (gx + gy) & 1;   // RB: colour of the own column's cell at z = 0
    const bool outp = threadIdx.y < NR && ly >= 1 && ly <= NR - 2 && gx < nx && gy < ny;
    const bool xrow = threadIdx.y < NR && (ly == 0 || ly == NR - 1);
    const int gyx = xrow ? (ly == 0 ? y0 - 2 : y0 + NR - 1) : gy;

    auto src = [](int c, int n, int per, int lo, int hi) {
        if (per) return ((c % n) + n) % n;
        return c < lo ? lo : (c > hi ? hi : c);
    };
    const int sy = g.st[1], sz = g.st[2];
    // Sigma and b: interior cells; rho, m and 1/rho: the first ghost layer is valid too
    const long long csig = (long long)(src(gy, ny, py, 0, ny - 1) + G) * sy + (src(gx, nx, px, 0, nx - 1) + G);
    const long long cir = (long long)(src(gy, ny, py, -1, ny) + G) * sy + (src(gx, nx, px, -1, nx) + G);
    const long long xsig = (long long)(src(gyx, ny, py, 0, ny - 1) + G) * sy + (src(gx, nx, px, 0, nx - 1) + G);
    const long long xir = (long long)(src(gyx, ny, py, -1, ny) + G) * sy + (src(gx, nx, px, -1, nx) + G);
    // every lane issues the same loads at clamped planes
    auto ldu = [&](long long o) { return F::template load_u<HASD>(U, D, o); };
    // plane index of a load: wrap (periodic z) or clamp, without a division
    // (P is within a few planes of the box)
    auto zsrc = [&](int c, int lo, int hi) {
        if (pz) {
            while (c < 0) c += nz;
            while (c >= nz) c -= nz;
            return c;
        }
        return c < lo ? lo : (c > hi ? hi : c);
    };
    auto load = [&](int P, PairIn<F, FIRST>& q) {
        const long long os = (long long)(zsrc(P, 0, nz - 1) + G) * sz;
        const long long oi = (long long)(zsrc(P, -1, nz) + G) * sz;
        q.s0 = F::load_s(Sin, os + csig);
        q.xs0 = F::load_s(Sin, os + xsig);
        if constexpr (FIRST) {
            q.rho = ldu(oi + cir);
            q.xrho = ldu(oi + xir);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                q.m[c] = ldu((1 + c) * fs + oi + cir);
                q.xm[c] = ldu((1 + c) * fs + oi + xir);
            }
            if constexpr (SPD) q.E = ldu(4 * fs + oi + cir);
        } else {
            q.b = b[os + csig];
            if constexpr (IRS) {
                q.ir = irs[oi + cir];
                q.xir = irs[oi + xir];
            } else {
                q.ir = ldu(oi + cir);
                q.xir = ldu(oi + xir);
            }
        }
    };
    auto inv = [](auto v) -> C {
        if constexpr (IRS && !FIRST)
            return v;
        else
            return fast_rcp(F::cvt(v));
    };

    const bool xlo = !px && gx == 0, xhi = !px && gx == nx - 1;
    const bool ylo = !py && gy == 0, yhi = !py && gy == ny - 1;
    const C alpha = C(g.alpha);
    const JacAxes<C> ja = jacobi_axes<C>(g);
    const int cx = lx + 2, cy = ly + 1;       // input-ring coordinates of the own column
    const int xr = ly == 0 ? 0 : NR + 1;      // input-ring row of the ring-2 row
    const int bxc = lx + 1;                   // b / level-1 column

    C qs1[2] = {C(0), C(0)};                  // level 1 at planes P-3, P-2
    // coefficients and source of the own cell at the plane level 1 formed
    // last (level 2 updates that cell one iteration later)
    JacCoef<C> kc = {C(0), C(0), C(0), C(0), C(0), C(0), C(0)};
    C bprev = C(0);
    C uq[3][3] = {};                          // FIRST: u of the own column at planes P-2, P-1, P
    double smax = 0.0;                        // SPD: CFL maximum of this thread's cells
    bool bad = false;

    // Ring slots follow r = (P - (z0 - 2)) mod 12, a compile-time constant
    // of each unrolled iteration: plane P goes to slot r mod 4 (Sigma, 1/rho)
    // and r mod 3 (b, u); level 1 at plane P-1 to slot (r+1) mod 2.
    auto iter = [&](int P, auto Rc, PairIn<F, FIRST>& slot) {
        constexpr int r = decltype(Rc)::value;
        // publish plane P, then refill the slot with plane P+PD
        constexpr int w4 = r % 4, w3 = r % 3;
        if constexpr (FIRST) {
            const C ir = inv(slot.rho);
            C u[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) u[c] = F::cvt(slot.m[c]) * ir;
            if (act) {
                ls0[w4][cy][cx] = F::cvt(slot.s0);
                lir[w4][cy][cx] = ir;
#pragma unroll
                for (int c = 0; c < 3; ++c) lu[c][w3][cy][cx] = u[c];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                uq[c][0] = uq[c][1];
                uq[c][1] = uq[c][2];
                uq[c][2] = u[c];
            }
            if (xrow) {
                const C xi = inv(slot.xrho);
                ls0[w4][xr][cx] = F::cvt(slot.xs0);
                lir[w4][xr][cx] = xi;
#pragma unroll
                for (int c = 0; c < 3; ++c) lu[c][w3][xr][cx] = F::cvt(slot.xm[c]) * xi;
            }
            if constexpr (SPD) {
                // every interior cell of the output tile, once per chunk plane
                if (outp && P >= z0 && P < z1)
                    smax = fmax(smax, cfl_speed(g, double(F::cvt(slot.rho)), double(F::cvt(slot.m[0])),
                                                double(F::cvt(slot.m[1])), double(F::cvt(slot.m[2])),
                                                double(F::cvt(slot.E)), bad));
            }
        } else {
            if (act) {
                ls0[w4][cy][cx] = F::cvt(slot.s0);
                lir[w4][cy][cx] = inv(slot.ir);
            }
            if (hasb) lb[w3][ly][bxc] = slot.b;
            if (xrow) {
                ls0[w4][xr][cx] = F::cvt(slot.xs0);
                lir[w4][xr][cx] = inv(slot.xir);
            }
        }
        load(min(P + PD, z1 + 1), slot);
        __syncthreads();
        if (P < z0) return;
        C v1 = C(0);
        const int z = P - 1;
        constexpr int a4 = (r + 3) % 4;   // plane P-1
        // level 1 at plane P-1.  Every lane evaluates it (all its LDS reads
        // are in bounds: rows 0..NR+1, columns 0..67 of the rings); lanes
        // that form no level-1 cell discard the result and only lev1 lanes
        // publish it.  Without a branch here the carried coefficients and
        // values need no per-lane merge (register moves) each plane.
        JacCoef<C> kn;
        C bn;
        {
            constexpr int m4 = (r + 2) % 4;   // plane P-2
            const C sc = ls0[a4][cy][cx];
            const C irv[6] = {lir[a4][cy][cx - 1], lir[a4][cy][cx + 1], lir[a4][cy - 1][cx], lir[a4][cy + 1][cx],
                              lir[m4][cy][cx], lir[w4][cy][cx]};
            const C sgv[6] = {face_or<NBSEL>(xlo, sc, &ls0[a4][cy][cx - 1]),
                              face_or<NBSEL>(xhi, sc, &ls0[a4][cy][cx + 1]),
                              face_or<NBSEL>(ylo, sc, &ls0[a4][cy - 1][cx]),
                              face_or<NBSEL>(yhi, sc, &ls0[a4][cy + 1][cx]),
                              face_or<NBSEL>(!pz && z == 0, sc, &ls0[m4][cy][cx]),
                              face_or<NBSEL>(!pz && z == nz - 1, sc, &ls0[w4][cy][cx])};
            kn = jacobi_coef(lir[a4][cy][cx], irv, ja);
            if constexpr (FIRST) {
                // source at this cell, eq. (9) left side
                constexpr int a3 = (r + 2) % 3;   // plane P-1
                C Gm[3][3];
                const C scx = C(0.5) * C(g.ih[0]), scy = C(0.5) * C(g.ih[1]), scz = C(0.5) * C(g.ih[2]);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Gm[c][0] = (lu[c][a3][cy][cx + 1] - lu[c][a3][cy][cx - 1]) * scx;
                    Gm[c][1] = (lu[c][a3][cy + 1][cx] - lu[c][a3][cy - 1][cx]) * scy;
                    Gm[c][2] = (uq[c][2] - uq[c][0]) * scz;
                }
                const C tr = Gm[0][0] + Gm[1][1] + Gm[2][2];
                C tr2 = C(0);
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int d = 0; d < 3; ++d) tr2 += Gm[c][d] * Gm[d][c];
                bn = alpha * (tr2 + tr * tr);
                if (outp && z >= z0 && z < z1) {
                    // b and (split form) 1/rho, face-ghost layer included, for the later passes
                    const long long o = (long long)(z + G) * sz + (long long)(gy + G) * sy + (gx + G);
                    b[o] = bn;
                    if constexpr (TAU) {
                        const C mu = C(mu_), lam = C(zeta_) - C(2) * C(mu_) / C(3);
#pragma unroll
                        for (int a = 0; a < 3; ++a)
#pragma unroll
                            for (int e = a; e < 3; ++e) {
                                C t = mu * (Gm[a][e] + Gm[e][a]);
                                if (a == e) t += lam * tr;
                                tau[(long long)tau_index(a, e) * fs + o] = t;
                            }
                    }
                    if constexpr (IRS) {
                        irs[o] = lir[a4][cy][cx];
                        if (gx == 0) irs[o - 1] = lir[a4][cy][cx - 1];
                        if (gx == nx - 1) irs[o + 1] = lir[a4][cy][cx + 1];
                        if (gy == 0) irs[o - sy] = lir[a4][cy - 1][cx];
                        if (gy == ny - 1) irs[o + sy] = lir[a4][cy + 1][cx];
                        if (z == 0) irs[o - sz] = lir[m4][cy][cx];
                        if (z == nz - 1) irs[o + sz] = lir[w4][cy][cx];
                    }
                }
            } else {
                bn = lb[(r + 2) % 3][ly][bxc];
            }
            v1 = jacobi_apply(bn, kn, sgv, ja);
            if constexpr (RB) v1 = ((par + z) & 1) ? sc : v1;   // black cells keep their value
            if (lev1) ls1[(r + 1) & 1][ly][bxc] = v1;
        }
        // level 2 (output) at plane P-2, with the coefficients and source
        // level 1 used there in the previous iteration
        if (outp && P >= z0 + 2) {
            const int z2 = P - 2;
            constexpr int a2 = r & 1;   // level 1 at plane P-2
            const C sc = qs1[1];
            const C sgv[6] = {face_or<NBSEL>(xlo, sc, &ls1[a2][ly][lx]),
                              face_or<NBSEL>(xhi, sc, &ls1[a2][ly][lx + 2]),
                              face_or<NBSEL>(ylo, sc, &ls1[a2][ly - 1][bxc]),
                              face_or<NBSEL>(yhi, sc, &ls1[a2][ly + 1][bxc]),
                              (!pz && z2 == 0) ? sc : qs1[0], (!pz && z2 == nz - 1) ? sc : v1};
            C v2 = jacobi_apply(bprev, kc, sgv, ja);
            if constexpr (RB) v2 = ((par + z2) & 1) ? v2 : sc;   // red cells keep level 1's value
            SS::store(Sout + (long long)(z2 + G) * sz + (long long)(gy + G) * sy + (gx + G), v2);
        }
        kc = kn;
        bprev = bn;
        qs1[0] = qs1[1];
        qs1[1] = v1;
    };

    PairIn<F, FIRST> pa, pb;
    load(z0 - 2, pa);
    load(z0 - 1, pb);
    // planes z0-2 .. z1+1, unrolled by 12 (the ring sizes' common multiple)
    // so that every ring slot is a constant; P is uniform, so the exit is
    // taken by the whole block
    int P = z0 - 2;
    const int Pend = z1 + 1;
    auto step = [&](auto Rc, PairIn<F, FIRST>& slot) {
        if (P > Pend) return false;
        iter(P, Rc, slot);
        ++P;
        return true;
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using I4 = std::integral_constant<int, 4>;
    using I5 = std::integral_constant<int, 5>;
    using I6 = std::integral_constant<int, 6>;
    using I7 = std::integral_constant<int, 7>;
    using I8 = std::integral_constant<int, 8>;
    using I9 = std::integral_constant<int, 9>;
    using I10 = std::integral_constant<int, 10>;
    using I11 = std::integral_constant<int, 11>;
    while (step(I0{}, pa) && step(I1{}, pb) && step(I2{}, pa) && step(I3{}, pb) && step(I4{}, pa) &&
           step(I5{}, pb) && step(I6{}, pa) && step(I7{}, pb) && step(I8{}, pa) && step(I9{}, pb) &&
           step(I10{}, pa) && step(I11{}, pb)) {
    }
    if constexpr (SPD) {
        for (int off = 32; off > 0; off >>= 1) smax = fmax(smax, __shfl_xor(smax, off, 64));
        if (threadIdx.x == 0) speed[(long long)blockIdx.x * (NR + 1) + threadIdx.y] = smax;
        if (bad) flag[0] = 1;
    }
}

}  // namespace igr
