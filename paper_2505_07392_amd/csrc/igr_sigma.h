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
    const C hx2 = C(g.ih[0]) * C(g.ih[0]), hy2 = C(g.ih[1]) * C(g.ih[1]), hz2 = C(g.ih[2]) * C(g.ih[2]);
    const C half = C(0.5);
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
            const C bxm = half * (ic + lr[slot][ey][exm]);
            const C bxp = half * (ic + lr[slot][ey][exp_]);
            const C bym = half * (ic + lr[slot][eym][ex]);
            const C byp = half * (ic + lr[slot][eyp][ex]);
            const C bzm = half * (ic + irR[2 + s]);
            const C bzp = half * (ic + irR[s]);
            C num = bR[s - 1];   // b at plane P-1-s (bR is shifted at the end of the iteration)
            C den = ic;
            num += alpha * (bxp * sxp + bxm * sxm) * hx2;
            den += alpha * (bxp + bxm) * hx2;
            num += alpha * (byp * syp + bym * sym) * hy2;
            den += alpha * (byp + bym) * hy2;
            num += alpha * (bzp * szp + bzm * szm) * hz2;
            den += alpha * (bzp + bzm) * hz2;
            newv[s] = num / den;
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

}  // namespace igr

namespace igr {

// One Jacobi sweep per pass, z-marching: a 64 x SWEEP_RY block of columns walks a
// chunk of z planes, keeping the z neighbours of Sigma and 1/rho in
// registers; x/y neighbours are read from memory (L1/L2 hits: adjacent
// lanes and rows).  Loads are issued ahead of use (see SweepCol) so that
// enough bytes are in flight per CU to cover HBM latency.  With FIRST the
// source b is formed in the same pass (from rho and m) and written for the
// later sweeps.  Per cell: FIRST reads rho, m, Sigma and writes Sigma, b;
// later sweeps read Sigma, rho, b and write Sigma.
// Loads of one iteration of the single-sweep kernel.  The own-column values
// of plane k+1 (which miss to HBM) are fetched PD iterations ahead; the x/y
// neighbours of plane k (mostly L1/L2 hits: other threads' columns) one
// iteration ahead.
template <class T, bool FIRST>
struct SweepCol {
    using C = typename Storage<T>::C;
    C rho, sig, b;      // rho, Sigma_in at plane k+1; b at plane k (later sweeps)
    C m[3];             // m at plane k+1 (FIRST)
};
template <class T, bool FIRST>
struct SweepNb {
    using C = typename Storage<T>::C;
    C rho[4], sig[4];   // x/y neighbours of plane k
    C m[4][3];          // (FIRST)
};

#ifndef IGR_SWEEP_RY
#define IGR_SWEEP_RY 4
#endif
constexpr int SWEEP_RY = IGR_SWEEP_RY;   // rows of a sweep block (64 x SWEEP_RY columns)

template <class T, bool FIRST>
__global__ __launch_bounds__(64 * SWEEP_RY) void k_sweep_z(const T* __restrict__ U, const T* __restrict__ Sin,
                                                 T* __restrict__ Sout, typename Storage<T>::C* __restrict__ b,
                                                 typename Storage<T>::C* __restrict__ irs, Geom g, int zc,
                                                 int tiles_x, int tiles_y) {
    using S = Storage<T>;
    using C = typename S::C;
    constexpr int PD = 3;   // own-column prefetch distance (planes)
    // FP64: the first sweep stores 1/rho (interior and the face-ghost layer)
    // and later sweeps read it instead of dividing again (same bytes as rho)
    constexpr bool IRS = sizeof(C) == 8;
    // 1-D grid in XCD-aware order: consecutive logical tiles (x fastest,
    // then y, then z chunk) run on one XCD, so rows shared by y-neighbour
    // tiles are fetched once into that XCD's L2
    int bidx = blockIdx.x;
    {
        constexpr int NXCD = 8;
        const int nb = gridDim.x;
        const int full = nb - nb % NXCD;
        if (bidx < full) bidx = (bidx % NXCD) * (full / NXCD) + bidx / NXCD;
    }
    const int bx = bidx % tiles_x;
    bidx /= tiles_x;
    const int by = bidx % tiles_y;
    const int bz = bidx / tiles_y;
    const int i = bx * 64 + threadIdx.x;
    const int j = by * SWEEP_RY + threadIdx.y;
    const int z0 = bz * zc;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    if (i >= nx || j >= ny) return;
    const int z1 = min(z0 + zc, nz);
    const long long fs = g.fs;
    const int sy = g.st[1], sz = g.st[2];
    const long long col = (long long)(j + G) * sy + (i + G);
    const C alpha = C(g.alpha);
    const C hx2 = C(g.ih[0]) * C(g.ih[0]), hy2 = C(g.ih[1]) * C(g.ih[1]), hz2 = C(g.ih[2]) * C(g.ih[2]);
    const C half = C(0.5);
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
    auto load_col = [&](int k, SweepCol<T, FIRST>& P) {   // for iteration k
        const long long op = zplane(k + 1);
        P.rho = (IRS && !FIRST) ? irs[op] : S::load(U + op);
        P.sig = S::load(Sin + col + (long long)(zsig(k + 1) + G) * sz);
        if (FIRST) {
#pragma unroll
            for (int c = 0; c < 3; ++c) P.m[c] = S::load(U + (1 + c) * fs + op);
        } else {
            P.b = b[zplane(k)];
        }
    };
    auto load_nb = [&](int k, SweepNb<T, FIRST>& P) {
        const long long o = zplane(k);
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            P.rho[n] = (IRS && !FIRST) ? irs[o + onb[n]] : S::load(U + o + onb[n]);
            P.sig[n] = S::load(Sin + o + osg[n]);
        }
        if (FIRST) {
#pragma unroll
            for (int n = 0; n < 4; ++n)
#pragma unroll
                for (int c = 0; c < 3; ++c) P.m[n][c] = S::load(U + (1 + c) * fs + o + onb[n]);
        }
    };
    auto inv_rho = [&](C v) { return (IRS && !FIRST) ? v : fast_rcp(v); };   // v: rho, or 1/rho stored
    C ir_m = (IRS && !FIRST) ? irs[zplane(z0 - 1)] : fast_rcp(S::load(U + zplane(z0 - 1)));
    C ir_c = (IRS && !FIRST) ? irs[zplane(z0)] : fast_rcp(S::load(U + zplane(z0)));
    C s_m = S::load(Sin + col + (long long)(zsig(z0 - 1) + G) * sz);
    C s_c = S::load(Sin + zplane(z0));
    C u_m[3], u_c[3];
    if (FIRST) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            u_m[c] = S::load(U + (1 + c) * fs + zplane(z0 - 1)) * ir_m;
            u_c[c] = S::load(U + (1 + c) * fs + zplane(z0)) * ir_c;
        }
    }
    SweepCol<T, FIRST> q[PD];   // own columns for iterations k .. k+PD-1
#pragma unroll
    for (int d = 0; d < PD; ++d)
        if (z0 + d < z1) load_col(z0 + d, q[d]);
    SweepNb<T, FIRST> cur, nxt;
    load_nb(z0, cur);
    for (int k = z0; k < z1; ++k) {
        const SweepCol<T, FIRST> cc = q[0];
#pragma unroll
        for (int d = 0; d < PD - 1; ++d) q[d] = q[d + 1];
        if (k + PD < z1) load_col(k + PD, q[PD - 1]);
        if (k + 1 < z1) load_nb(k + 1, nxt);
        const long long o = zplane(k);
        const C ir_p = inv_rho(cc.rho);
        const C s_p = cc.sig;
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
            for (int c = 0; c < 3; ++c) u_p[c] = cc.m[c] * ir_p;
            C Gm[3][3];
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                const C sc = C(0.5) * C(g.ih[d]);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    Gm[c][d] = (cur.m[2 * d + 1][c] * irn[2 * d + 1] - cur.m[2 * d][c] * irn[2 * d]) * sc;
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
        } else {
            bk = cc.b;
        }
        const C ic = ir_c;
        const C bxm = half * (ic + irn[0]);
        const C bxp = half * (ic + irn[1]);
        const C bym = half * (ic + irn[2]);
        const C byp = half * (ic + irn[3]);
        const C bzm = half * (ic + ir_m);
        const C bzp = half * (ic + ir_p);
        C num = bk;
        C den = ic;
        num += alpha * (bxp * cur.sig[1] + bxm * cur.sig[0]) * hx2;
        den += alpha * (bxp + bxm) * hx2;
        num += alpha * (byp * cur.sig[3] + bym * cur.sig[2]) * hy2;
        den += alpha * (byp + bym) * hy2;
        num += alpha * (bzp * s_p + bzm * s_m) * hz2;
        den += alpha * (bzp + bzm) * hz2;
        S::store(Sout + o, num * fast_rcp(den));
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

}  // namespace igr
