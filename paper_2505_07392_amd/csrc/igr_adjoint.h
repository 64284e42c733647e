// Hand-written discrete adjoint (vector-Jacobian product) of one IGR
// right-hand side and of the SSP-RK3 step, FP64.
//
// Forward pieces and their transposes (all gather form, no atomics):
//   ghosts of U         -> k_adj_bc_state     ghost cotangents folded into the
//                                             copied interior cells and into
//                                             the jet-disc states
//   source b(U)         -> k_adj_source       via G_ij and u = m / rho
//   Jacobi sweep        -> k_adj_jac1/2       level by level, using the stored
//                                             iterates (the sweep is linear in
//                                             Sigma, nonlinear in rho)
//   Sigma ghosts        -> k_adj_sigma_bc
//   reconstruction+LLF  -> k_adj_face (per face) + k_adj_recon_gather (per
//                          cell, transposed stencil)
// The LLF maximum sends the wave-speed cotangent to the larger side (half
// to each on a tie) and |u_n| uses sign(u_n) (0 at 0), matching the
// conventions of reverse-mode differentiation of max and abs.
#pragma once

#include "igr_kernels.h"

namespace igr {

// Cell index along axis d of the interior cell that padded index p copies
// (periodic wrap or clamp), for Sigma and for U outside inflow columns.
__device__ __forceinline__ int ghost_source(int p, int n, int periodic) {
    if (periodic) return ((p % n) + n) % n;
    return p < 0 ? 0 : (p > n - 1 ? n - 1 : p);
}

// Transverse axes of axis d and a thread's (a, b, along-d) decomposition.
struct Line {
    int a, b;
};
__device__ __forceinline__ Line transverse(int d) {
    Line L;
    L.a = d == 0 ? 1 : 0;
    L.b = d == 2 ? 1 : 2;
    return L;
}

// ---------------------------------------------------------------------------
// Flux: per face, reverse of reconstruction + LLF.  Face l+1/2 (l = -1..n-1)
// is stored at padded position l+1 along d of the 12 face arrays FA:
// [0..4] UL-bar, [5..9] UR-bar, [10] SL-bar, [11] SR-bar.
// ---------------------------------------------------------------------------

struct SideFwd {
    double rho, m[3], E, S;
    double ir, p, un, c, s;
};

__device__ __forceinline__ void side_forward(SideFwd& v, int d, double gamma) {
    v.ir = 1.0 / v.rho;
    v.p = (gamma - 1.0) * (v.E - 0.5 * (v.m[0] * v.m[0] + v.m[1] * v.m[1] + v.m[2] * v.m[2]) * v.ir);
    v.un = v.m[d] * v.ir;
    v.c = sqrt(gamma * v.p * v.ir);
    v.s = fabs(v.un) + v.c;
}

// Reverse of one side given the cotangents of un, p, S-free terms, s.
// Inputs: unb, pb, sb (wave-speed cotangent); accumulates into Ub[5].
__device__ __forceinline__ void side_reverse(const SideFwd& v, int d, double gamma, double unb, double pb, double sb,
                                             double Ub[5]) {
    // s = |un| + c
    const double sgn = v.un > 0.0 ? 1.0 : (v.un < 0.0 ? -1.0 : 0.0);
    unb += sb * sgn;
    const double cb = sb;
    // c = sqrt(gamma p ir)
    double irb = 0.0;
    if (cb != 0.0) {
        const double t = cb / (2.0 * v.c);
        pb += t * gamma * v.ir;
        irb += t * gamma * v.p;
    }
    // un = m_d ir
    Ub[1 + d] += unb * v.ir;
    irb += unb * v.m[d];
    // p = (gamma-1)(E - 0.5 |m|^2 ir)
    const double g1 = gamma - 1.0;
    Ub[4] += g1 * pb;
    for (int k = 0; k < 3; ++k) Ub[1 + k] -= g1 * pb * v.m[k] * v.ir;
    irb -= g1 * pb * 0.5 * (v.m[0] * v.m[0] + v.m[1] * v.m[1] + v.m[2] * v.m[2]);
    // ir = 1/rho
    Ub[0] -= irb * v.ir * v.ir;
}

template <int D, int ORDER>
__global__ __launch_bounds__(256) void k_adj_face(const double* __restrict__ U, const double* __restrict__ Sg,
                                                  const double* __restrict__ Lb, double* __restrict__ FA, Geom g) {
    const Line tl = transverse(D);
    const int nd = g.n[D];
    const long long nlines = (long long)g.n[tl.a] * g.n[tl.b];
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nlines * (nd + 1)) return;
    const int f = int(t % (nd + 1));          // face index: face l+1/2 with l = f-1
    const long long line = t / (nd + 1);
    const int ia = int(line % g.n[tl.a]);
    const int ib = int(line / g.n[tl.a]);
    const int sd = g.st[D];
    const long long base = (long long)(ia + G) * g.st[tl.a] + (long long)(ib + G) * g.st[tl.b];
    const int l = f - 1;
    const long long ol = base + (long long)(l + G) * sd;   // left cell of the face
    const double gamma = g.gamma;
    // face flux cotangent from the two adjacent cells' L-bar
    double Fb[5];
    for (int k = 0; k < 5; ++k) {
        const double right = (l + 1 <= nd - 1) ? Lb[k * g.fs + ol + sd] : 0.0;
        const double left = (l >= 0) ? Lb[k * g.fs + ol] : 0.0;
        Fb[k] = (right - left) * g.ih[D];
    }
    // forward: reconstruct
    double q[6][6];
    for (int p = 0; p < 6; ++p) {
        const long long op = ol + (long long)(p - 2) * sd;
        for (int k = 0; k < 5; ++k) q[k][p] = U[k * g.fs + op];
        q[5][p] = Sg[op];
    }
    SideFwd L, R;
    double UL[5], UR[5];
    // cells l-2..l+3 in q[.][0..5]; third order reads l-1..l+2
    auto rec = [&](const double (&v)[6], double& l, double& r) {
        if constexpr (ORDER == 5) {
            l = recon_left(v[0], v[1], v[2], v[3], v[4]);
            r = recon_right(v[1], v[2], v[3], v[4], v[5]);
        } else {
            l = recon3_left(v[1], v[2], v[3]);
            r = recon3_right(v[2], v[3], v[4]);
        }
    };
    for (int k = 0; k < 5; ++k) rec(q[k], UL[k], UR[k]);
    L.rho = UL[0];
    R.rho = UR[0];
    for (int k = 0; k < 3; ++k) {
        L.m[k] = UL[1 + k];
        R.m[k] = UR[1 + k];
    }
    L.E = UL[4];
    R.E = UR[4];
    rec(q[5], L.S, R.S);
    side_forward(L, D, gamma);
    side_forward(R, D, gamma);
    const double lam = fmax(L.s, R.s);
    // reverse of F = 1/2 (F_L + F_R) - 1/2 lam (UR - UL)
    double ULb[5] = {0, 0, 0, 0, 0}, URb[5] = {0, 0, 0, 0, 0};
    double lamb = 0.0;
    for (int k = 0; k < 5; ++k) {
        lamb -= 0.5 * Fb[k] * (UR[k] - UL[k]);
        ULb[k] += 0.5 * lam * Fb[k];
        URb[k] -= 0.5 * lam * Fb[k];
    }
    double unbL = 0.0, unbR = 0.0, pbL = 0.0, pbR = 0.0, SbL = 0.0, SbR = 0.0;
    // mass: 1/2 (mL_d + mR_d)
    ULb[1 + D] += 0.5 * Fb[0];
    URb[1 + D] += 0.5 * Fb[0];
    // momentum: 1/2 (m_k un + delta_kd (p + S)) per side
    for (int k = 0; k < 3; ++k) {
        ULb[1 + k] += 0.5 * Fb[1 + k] * L.un;
        URb[1 + k] += 0.5 * Fb[1 + k] * R.un;
        unbL += 0.5 * Fb[1 + k] * L.m[k];
        unbR += 0.5 * Fb[1 + k] * R.m[k];
    }
    pbL += 0.5 * Fb[1 + D];
    pbR += 0.5 * Fb[1 + D];
    SbL += 0.5 * Fb[1 + D];
    SbR += 0.5 * Fb[1 + D];
    // energy: 1/2 (E + p + S) un per side
    ULb[4] += 0.5 * Fb[4] * L.un;
    URb[4] += 0.5 * Fb[4] * R.un;
    pbL += 0.5 * Fb[4] * L.un;
    pbR += 0.5 * Fb[4] * R.un;
    SbL += 0.5 * Fb[4] * L.un;
    SbR += 0.5 * Fb[4] * R.un;
    unbL += 0.5 * Fb[4] * (L.E + L.p + L.S);
    unbR += 0.5 * Fb[4] * (R.E + R.p + R.S);
    // lam = max(sL, sR)
    const double wl = L.s > R.s ? 1.0 : (L.s == R.s ? 0.5 : 0.0);
    side_reverse(L, D, gamma, unbL, pbL, lamb * wl, ULb);
    side_reverse(R, D, gamma, unbR, pbR, lamb * (1.0 - wl), URb);
    const long long of = base + (long long)(f + G) * sd;   // face storage position
    for (int k = 0; k < 5; ++k) {
        FA[k * g.fs + of] = ULb[k];
        FA[(5 + k) * g.fs + of] = URb[k];
    }
    FA[10 * g.fs + of] = SbL;
    FA[11 * g.fs + of] = SbR;
}

// Transposed reconstruction: padded cell q along D (q = -3..n+2) gathers
// from the faces whose stencils contain it; adds into Ub (5) and Sb.
// Fifth order: the left state of face l+1/2 weighs cells l-2..l+2 by
// (2, -13, 47, 27, -3)/60, the right state l-1..l+3 by the mirror image;
// third order: l-1..l+1 by (-1, 5, 2)/6 and l..l+2 by (2, 5, -1)/6.
template <int D, int ORDER>
__global__ __launch_bounds__(256) void k_adj_recon_gather(const double* __restrict__ FA, double* __restrict__ Ub,
                                                          double* __restrict__ Sb, Geom g) {
    const Line tl = transverse(D);
    const int nd = g.n[D];
    const int np = nd + 2 * G;
    const long long nlines = (long long)g.n[tl.a] * g.n[tl.b];
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nlines * np) return;
    const int qp = int(t % np) - G;   // padded index along D
    const long long line = t / np;
    const int ia = int(line % g.n[tl.a]);
    const int ib = int(line / g.n[tl.a]);
    const int sd = g.st[D];
    const long long base = (long long)(ia + G) * g.st[tl.a] + (long long)(ib + G) * g.st[tl.b];
    constexpr int NS = ORDER == 5 ? 5 : 3;                 // cells per one-sided stencil
    constexpr int SL = ORDER == 5 ? 2 : 1;                 // left state: cells l-SL .. l-SL+NS-1
    constexpr int SR = ORDER == 5 ? 1 : 0;                 // right state: cells l-SR ..
    constexpr double DEN = ORDER == 5 ? 60.0 : 6.0;
    const double CLc[5] = {ORDER == 5 ? 2.0 : -1.0, ORDER == 5 ? -13.0 : 5.0, ORDER == 5 ? 47.0 : 2.0, 27.0, -3.0};
    const double CRc[5] = {ORDER == 5 ? -3.0 : 2.0, ORDER == 5 ? 27.0 : 5.0, ORDER == 5 ? 47.0 : -1.0, -13.0, 2.0};
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int m = 0; m < NS; ++m) {
        // left state of face l: cell qp = l - SL + m
        const int lL = qp + SL - m;
        if (lL >= -1 && lL <= nd - 1) {
            const long long of = base + (long long)(lL + 1 + G) * sd;
            const double w = CLc[m] / DEN;
            for (int k = 0; k < 5; ++k) acc[k] += w * FA[k * g.fs + of];
            acc[5] += w * FA[10 * g.fs + of];
        }
        // right state of face l: cell qp = l - SR + m
        const int lR = qp + SR - m;
        if (lR >= -1 && lR <= nd - 1) {
            const long long of = base + (long long)(lR + 1 + G) * sd;
            const double w = CRc[m] / DEN;
            for (int k = 0; k < 5; ++k) acc[k] += w * FA[(5 + k) * g.fs + of];
            acc[5] += w * FA[11 * g.fs + of];
        }
    }
    const long long oc = base + (long long)(qp + G) * sd;
    for (int k = 0; k < 5; ++k) Ub[k * g.fs + oc] += acc[k];
    Sb[oc] += acc[5];
}

// Sigma ghosts transposed: interior cell c gathers the cotangents of the
// face-ghost positions that copy it; out = Sig_bar_in + Sb(interior) + folds.
__global__ __launch_bounds__(256) void k_adj_sigma_bc(const double* __restrict__ Sb, const double* __restrict__ Sin,
                                                      double* __restrict__ Sout, Geom g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const int idx[3] = {i, j, k};
    const long long o = cell_offset(g, i, j, k);
    double v = Sin[o] + Sb[o];
    for (int d = 0; d < 3; ++d) {
        const int n = g.n[d];
        for (int gidx = 0; gidx < 2 * G; ++gidx) {
            const int p = gidx < G ? -1 - gidx : n + (gidx - G);
            if (ghost_source(p, n, g.periodic[d]) == idx[d]) v += Sb[o + (long long)(p - idx[d]) * g.st[d]];
        }
    }
    Sout[o] = v;
}

// ---------------------------------------------------------------------------
// Jacobi sweep adjoint.  Sigma^k_c = N_c / D_c with
//   N_c = b_c + alpha sum_nb beta_{c,nb} S_nb / h^2,
//   D_c = ir_c + alpha sum_nb beta_{c,nb} / h^2,  beta = (ir_c + ir_nb)/2.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double jac_den(const double* ir, long long o, const Geom& g) {
    const double ic = ir[o];
    double den = ic;
    for (int d = 0; d < 3; ++d) {
        const double h2 = g.ih[d] * g.ih[d];
        const double bp = 0.5 * (ic + ir[o + g.st[d]]);
        const double bm = 0.5 * (ic + ir[o - g.st[d]]);
        den += g.alpha * (bp + bm) * h2;
    }
    return den;
}

// N-bar = Sig-bar^k / D, D-bar = -N-bar Sigma^k; b-bar += N-bar.
__global__ __launch_bounds__(256) void k_adj_jac1(const double* __restrict__ Sbk, const double* __restrict__ Sk,
                                                  const double* __restrict__ ir, double* __restrict__ Nb,
                                                  double* __restrict__ Db, double* __restrict__ bb, Geom g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const long long o = cell_offset(g, i, j, k);
    const double den = jac_den(ir, o, g);
    const double nb = Sbk[o] / den;
    Nb[o] = nb;
    Db[o] = -nb * Sk[o];
    bb[o] += nb;
}

// Sig-bar^{k-1} (interior) and ir-bar (interior and face ghosts) by gather.
// Skm1 = Sigma^{k-1} (interior; ghosts are not read: the sweep maps a
// missing neighbour to the wrapped cell or to the cell itself).
//   ir-bar_q  = [q interior] (D-bar_q + sum_slots beta-bar_{q,slot}/2)
//             + sum over equations e with e + s e_d = q of beta-bar_{e,d,s}/2
//   beta-bar_{e,d,s} = alpha/h_d^2 (N-bar_e S_{src(e,d,s)} + D-bar_e)
//   Sig-bar^{k-1}_c = sum over (e,d,s) with src(e,d,s) = c of
//                     N-bar_e alpha beta_{e,d,s}/h_d^2
__global__ __launch_bounds__(256) void k_adj_jac2(const double* __restrict__ Nb, const double* __restrict__ Db,
                                                  const double* __restrict__ Skm1, const double* __restrict__ ir,
                                                  double* __restrict__ Sbkm1, double* __restrict__ irb, Geom g) {
    const int pi = blockIdx.x * blockDim.x + threadIdx.x - G;
    const int pj = blockIdx.y * blockDim.y + threadIdx.y - G;
    const int pk = blockIdx.z - G;
    if (pi >= g.n[0] + G || pj >= g.n[1] + G) return;
    const int pidx[3] = {pi, pj, pk};
    int outside = 0;
    for (int d = 0; d < 3; ++d) outside += (pidx[d] < 0 || pidx[d] >= g.n[d]);
    if (outside > 1) return;
    const bool interior = outside == 0;
    const long long o = (long long)(pk + G) * g.st[2] + (long long)(pj + G) * g.st[1] + (pi + G);
    const double alpha = g.alpha;
    double irb_acc = 0.0;
    if (interior) {
        const double nbc = Nb[o], dbc = Db[o];
        irb_acc += dbc;
        for (int d = 0; d < 3; ++d) {
            const double h2 = g.ih[d] * g.ih[d];
            for (int s = -1; s <= 1; s += 2) {
                const int src = ghost_source(pidx[d] + s, g.n[d], g.periodic[d]);
                const double Snb = Skm1[o + (long long)(src - pidx[d]) * g.st[d]];
                irb_acc += 0.5 * alpha * h2 * (nbc * Snb + dbc);
            }
        }
    }
    for (int d = 0; d < 3; ++d) {
        const double h2 = g.ih[d] * g.ih[d];
        for (int s = -1; s <= 1; s += 2) {
            int e[3] = {pidx[0], pidx[1], pidx[2]};
            e[d] -= s;   // e + s e_d = q
            bool e_in = true;
            for (int a = 0; a < 3; ++a) e_in = e_in && e[a] >= 0 && e[a] < g.n[a];
            if (!e_in) continue;
            const long long oe = o - (long long)s * g.st[d];
            const int src = ghost_source(e[d] + s, g.n[d], g.periodic[d]);
            const double Snb = Skm1[oe + (long long)(src - e[d]) * g.st[d]];
            irb_acc += 0.5 * alpha * h2 * (Nb[oe] * Snb + Db[oe]);
        }
    }
    irb[o] += irb_acc;
    if (!interior) return;
    double sb = 0.0;
    for (int d = 0; d < 3; ++d) {
        const int n = g.n[d];
        const int c = pidx[d];
        const double h2 = g.ih[d] * g.ih[d];
        for (int s = -1; s <= 1; s += 2) {
            const int cand[4] = {c - s, c - s + n, c - s - n, c};
            for (int t = 0; t < 4; ++t) {
                const int ed = cand[t];
                if (ed < 0 || ed >= n) continue;
                bool dup = false;
                for (int u = 0; u < t; ++u) dup = dup || cand[u] == ed;
                if (dup) continue;
                if (ghost_source(ed + s, n, g.periodic[d]) != c) continue;
                const long long oe = o + (long long)(ed - c) * g.st[d];
                const double beta = 0.5 * (ir[oe] + ir[oe + (long long)s * g.st[d]]);
                sb += Nb[oe] * alpha * beta * h2;
            }
        }
    }
    Sbkm1[o] = sb;
}

// ---------------------------------------------------------------------------
// Source adjoint: b = alpha (sum_ij G_ij G_ji + tr^2), G_ij = (u_i(+e_j) -
// u_i(-e_j)) / (2 h_j).  Padded positions (interior + face ghosts) gather
// u-bar, then m-bar = u-bar ir and ir-bar += u-bar . m.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void grad_u(const double* U, const double* ir, long long o, const Geom& g,
                                       double Gm[3][3]) {
    for (int j = 0; j < 3; ++j) {
        const long long op = o + g.st[j], om = o - g.st[j];
        for (int c = 0; c < 3; ++c) {
            const double up = U[(1 + c) * g.fs + op] * ir[op];
            const double um = U[(1 + c) * g.fs + om] * ir[om];
            Gm[c][j] = (up - um) * (0.5 * g.ih[j]);
        }
    }
}

__global__ __launch_bounds__(256) void k_adj_source(const double* __restrict__ U, const double* __restrict__ ir,
                                                    const double* __restrict__ bb, double* __restrict__ Ub,
                                                    double* __restrict__ irb, Geom g) {
    const int pi = blockIdx.x * blockDim.x + threadIdx.x - G;
    const int pj = blockIdx.y * blockDim.y + threadIdx.y - G;
    const int pk = blockIdx.z - G;
    if (pi >= g.n[0] + G || pj >= g.n[1] + G) return;
    const int pidx[3] = {pi, pj, pk};
    int outside = 0;
    for (int d = 0; d < 3; ++d) outside += (pidx[d] < 0 || pidx[d] >= g.n[d]);
    if (outside > 1) return;
    const long long o = (long long)(pk + G) * g.st[2] + (long long)(pj + G) * g.st[1] + (pi + G);
    double ub[3] = {0, 0, 0};
    for (int j = 0; j < 3; ++j) {
        for (int s = -1; s <= 1; s += 2) {
            int eidx[3] = {pidx[0], pidx[1], pidx[2]};
            eidx[j] += s;   // e = position + s e_j; position is e's (-s) neighbour
            bool e_in = true;
            for (int a = 0; a < 3; ++a) e_in = e_in && eidx[a] >= 0 && eidx[a] < g.n[a];
            if (!e_in) continue;
            const long long oe = o + (long long)s * g.st[j];
            const double be = bb[oe];
            if (be == 0.0) continue;
            double Gm[3][3];
            grad_u(U, ir, oe, g, Gm);
            const double tr = Gm[0][0] + Gm[1][1] + Gm[2][2];
            for (int c = 0; c < 3; ++c) {
                const double Gb = be * g.alpha * (2.0 * Gm[j][c] + (c == j ? 2.0 * tr : 0.0));
                // G_cj(e) = (u_c(e + e_j) - u_c(e - e_j)) ih_j / 2; position = e - s e_j
                ub[c] += -double(s) * Gb * 0.5 * g.ih[j];
            }
        }
    }
    double irb_acc = 0.0;
    for (int c = 0; c < 3; ++c) {
        Ub[(1 + c) * g.fs + o] += ub[c] * ir[o];
        irb_acc += ub[c] * U[(1 + c) * g.fs + o];
    }
    irb[o] += irb_acc;
}

// ir = 1/rho on padded positions (interior + face ghosts) of a filled U.
__global__ __launch_bounds__(256) void k_inv_rho(const double* __restrict__ U, double* __restrict__ ir, Geom g) {
    const int pi = blockIdx.x * blockDim.x + threadIdx.x - G;
    const int pj = blockIdx.y * blockDim.y + threadIdx.y - G;
    const int pk = blockIdx.z - G;
    if (pi >= g.n[0] + G || pj >= g.n[1] + G) return;
    const int pidx[3] = {pi, pj, pk};
    int outside = 0;
    for (int d = 0; d < 3; ++d) outside += (pidx[d] < 0 || pidx[d] >= g.n[d]);
    if (outside > 1) return;
    const long long o = (long long)(pk + G) * g.st[2] + (long long)(pj + G) * g.st[1] + (pi + G);
    ir[o] = 1.0 / U[o];
}

// rho-bar += -ir-bar ir^2 on padded positions.
__global__ __launch_bounds__(256) void k_adj_irho(const double* __restrict__ ir, const double* __restrict__ irb,
                                                  double* __restrict__ Ub, Geom g) {
    const int pi = blockIdx.x * blockDim.x + threadIdx.x - G;
    const int pj = blockIdx.y * blockDim.y + threadIdx.y - G;
    const int pk = blockIdx.z - G;
    if (pi >= g.n[0] + G || pj >= g.n[1] + G) return;
    const int pidx[3] = {pi, pj, pk};
    int outside = 0;
    for (int d = 0; d < 3; ++d) outside += (pidx[d] < 0 || pidx[d] >= g.n[d]);
    if (outside > 1) return;
    const long long o = (long long)(pk + G) * g.st[2] + (long long)(pj + G) * g.st[1] + (pi + G);
    Ub[o] -= irb[o] * ir[o] * ir[o];
}

// Ghosts of U transposed: interior cell c receives its own cotangent plus
// those of the face ghosts copying it ((1-chi) of them on x-min inflow
// columns).  Writes Uout (interior, 5 fields); `jetcol` gets, per x-min
// column (k*ny + j) of an inflow owner, chi * sum of its ghost cotangents.
__global__ __launch_bounds__(256) void k_adj_bc_state(const double* __restrict__ Ub, double* __restrict__ Uout,
                                                      const int* __restrict__ owner, const double* __restrict__ chi,
                                                      double* __restrict__ jetcol, Geom g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const int idx[3] = {i, j, k};
    const long long o = cell_offset(g, i, j, k);
    const int q = owner ? owner[(long long)k * g.n[1] + j] : -1;
    const double c = q >= 0 ? chi[(long long)k * g.n[1] + j] : 0.0;
    for (int f = 0; f < 5; ++f) {
        const double* F = Ub + f * g.fs;
        double v = F[o];
        for (int d = 0; d < 3; ++d) {
            const int n = g.n[d];
            for (int gi = 0; gi < 2 * G; ++gi) {
                const int p = gi < G ? -1 - gi : n + (gi - G);
                if (ghost_source(p, n, g.periodic[d]) != idx[d]) continue;
                double w = 1.0;
                if (d == 0 && p < 0 && q >= 0) w = 1.0 - c;
                v += w * F[o + (long long)(p - idx[d]) * g.st[d]];
            }
        }
        Uout[f * g.fs + o] = v;
        if (i == 0 && q >= 0 && jetcol) {
            double s = 0.0;
            for (int l = 1; l <= G; ++l) s += F[o - (long long)l * g.st[0]];
            jetcol[((long long)k * g.n[1] + j) * 5 + f] = c * s;
        }
    }
}

// y = a x + b y on interior cells of nf fields (padded layout).
__global__ __launch_bounds__(256) void k_axpby(double a, const double* __restrict__ x, double b, double* y, int nf,
                                               Geom g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const long long o = cell_offset(g, i, j, k);
    for (int f = 0; f < nf; ++f) {
        const long long of = f * g.fs + o;
        y[of] = a * (x ? x[of] : 0.0) + b * y[of];
    }
}

}  // namespace igr
