// Viscous terms of the Navier-Stokes balances, eqs. (2)-(3), with the
// stress of eq. (5): tau = mu (G + G^T) + (zeta - 2 mu / 3) tr(G) I,
// G_ij = d u_i / d x_j.  They are added to a right-hand side or RK stage
// that the inviscid flux kernel has already written ("sequential summation
// of right-hand side contributions"):
//
//   k_stress          tau at interior cells from G by second-order central
//                     differences of u = m / rho (the paper: second-order
//                     derivatives of u suffice).  tau is symmetric: six
//                     stored components (xx, xy, xz, yy, yz, zz).  Their
//                     ghost cells follow Sigma's rule (k_bc_sigma per
//                     component; that rule copies values, so it commutes
//                     with the linear map G -> tau);
//   k_viscous_tiled   per face of direction d, the viscous flux: each
//                     side's tau e_d reconstructed from the cell-centre
//                     stresses with the weights of the conserved variables
//                     (Algorithm 1 reconstructs the gradients with the same
//                     coefficients; tau is linear in G), each side's
//                     velocity from the reconstructed conserved variables,
//                     and the mean of the two sides' fluxes -tau e_d
//                     (momenta) and -(u . tau) e_d (energy); each cell's
//                     divergence is scaled by the stage's weight of dt and
//                     added to the output.
//
// k_viscous_tiled follows the flux kernel's layout: a block owns a 64 x TY
// tile of the x-y plane and marches through a chunk of z planes.  The
// column's seven z-stencil fields (rho, m, tau_xz, tau_yz, tau_zz) of
// planes k-2..k+3 sit in a register queue; plane k's nine in-plane fields
// (rho, m, tau_xx, tau_xy, tau_xz, tau_yy, tau_yz) with a three-cell halo
// are staged in LDS for the x and y stencils.  Every face is computed
// once: x faces i+1/2 and y faces j+1/2 by the tile's own waves, the tile's
// left x faces and lower y faces by one extra wave, the z face k+1/2 from
// the queue (face k-1/2 is kept from the previous plane); x/y face fluxes
// go through LDS.  A tile's own columns are read from HBM once; its
// in-plane halo is read again by the neighbouring tiles (about 1.4-1.5x
// the compulsory bytes in all), where a kernel that reads every stencil
// from global memory would fetch each z stencil seven times.
#pragma once

#include "igr_adjoint.h"
#include "igr_flux.h"

namespace igr {

// A block owns a 64 x TY tile of the x-y plane and marches a chunk of z
// planes: rho and m of planes k-1, k, k+1 of its columns stay in a register
// queue (plane k+2 is fetched one iteration ahead), plane k with a one-cell
// halo is staged in LDS for the x and y differences (the halo of plane k+1
// is fetched while plane k is processed), so that each input value is read
// from HBM about once.
constexpr int STRESS_TX = 64;
template <class F, int TY, bool HASD>
__global__ __launch_bounds__(STRESS_TX* TY) void k_stress(const typename F::TB* __restrict__ U,
                                                          const typename F::TD* __restrict__ D,
                                                          typename F::C* __restrict__ T6, Geom g, double mu_,
                                                          double zeta_, int tiles_x, int tiles_y, int zc) {
    using C = typename F::C;
    constexpr int TX = STRESS_TX;
    static_assert(TX * TY <= 1024, "at most 1024 threads per block");
    __shared__ C pl[4][TY + 2][TX + 2];
    const int lane = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int tid = wv * TX + lane;
    int tx, ty, cz;
    tile_coords(xcd_remap(blockIdx.x, gridDim.x), tiles_x, tiles_y, tx, ty, cz);
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = cz * zc;
    const int z1 = min(z0 + zc, nz);
    const long long fs = g.fs;
    const int sy = g.st[1], sz = g.st[2];
    const int i = x0 + lane, j = y0 + wv;
    // cells up to n (the last interior cell's + neighbour) are loaded
    const bool col_load = i < nx + 1 && j < ny + 1;
    const bool col_out = i < nx && j < ny;
    const uint32_t col = uint32_t((j + G) * sy + (i + G));
    // the stage input (U, + its difference D in the split form's later stages)
    auto ld = [&](int f, int plane, uint32_t o) -> C {
        plane = __builtin_amdgcn_readfirstlane(plane);
        const long long po = (long long)f * fs + (long long)(plane + G) * sz;
        return F::cvt(F::template load_up<HASD>(U + po, HASD ? D + po : nullptr, o));
    };
    // rho, m_x, m_y, m_z of planes k-1 (qm), k (q0), k+1 (qp), k+2 (nxt)
    // after the shift at the top of iteration k
    C qm[4], q0[4], qp[4], nxt[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) qm[f] = q0[f] = qp[f] = nxt[f] = f == 0 ? C(1) : C(0);
    if (col_load) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            q0[f] = ld(f, z0 - 1, col);
            qp[f] = ld(f, z0, col);
            nxt[f] = ld(f, z0 + 1, col);
        }
    }
    // one-cell halo: the y rows (2 rows x TX columns x 4 fields) row by row
    // to the waves, the x columns (2 x TY x 4) to the first 8 TY threads
    constexpr int NYR = 4 * 2;
    constexpr int HY = (NYR + TY - 1) / TY;
    constexpr int NXH = 4 * 2 * TY;
    C hy[HY], hx = C(0);
    auto y_slot = [&](int s, int& f, int& cy) -> bool {
        const int rf = wv + s * TY;
        if (rf >= NYR) return false;
        f = rf >> 1;
        cy = (rf & 1) ? TY : -1;
        const int gy = y0 + cy;
        return i < nx + 1 && gy >= -1 && gy < ny + 1;
    };
    auto x_slot = [&](int& f, int& cx, int& cy) -> bool {
        if (tid >= NXH) return false;
        f = tid / (2 * TY);
        const int r = tid - f * 2 * TY;
        cy = r >> 1;
        cx = (r & 1) ? TX : -1;
        const int gx = x0 + cx;
        return gx >= -1 && gx < nx + 1 && y0 + cy < ny + 1;
    };
    auto load_halo = [&](int plane) {
#pragma unroll
        for (int s = 0; s < HY; ++s) {
            int f, cy;
            hy[s] = C(0);
            if (y_slot(s, f, cy)) hy[s] = ld(f, plane, uint32_t((y0 + cy + G) * sy + (i + G)));
        }
        int f, cx, cy;
        hx = C(0);
        if (x_slot(f, cx, cy)) hx = ld(f, plane, uint32_t((y0 + cy + G) * sy + (x0 + cx + G)));
    };
    load_halo(z0);
    const C mu = C(mu_), lam = C(zeta_) - C(2) * C(mu_) / C(3);
    const C scx = C(0.5) * C(g.ih[0]), scy = C(0.5) * C(g.ih[1]), scz = C(0.5) * C(g.ih[2]);
    for (int k = z0; k < z1; ++k) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            qm[f] = q0[f];
            q0[f] = qp[f];
            qp[f] = nxt[f];
        }
        // plane k+2 exists (ghost layers reach nz+2) while k+1 < z1
        if (col_load && k + 1 < z1) {
#pragma unroll
            for (int f = 0; f < 4; ++f) nxt[f] = ld(f, k + 2, col);
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) pl[f][wv + 1][lane + 1] = q0[f];
#pragma unroll
        for (int s = 0; s < HY; ++s) {
            int f, cy;
            if (y_slot(s, f, cy)) pl[f][cy + 1][lane + 1] = hy[s];
        }
        {
            int f, cx, cy;
            if (x_slot(f, cx, cy)) pl[f][cy + 1][cx + 1] = hx;
        }
        if (k + 1 < z1) load_halo(k + 1);
        __syncthreads();
        if (col_out) {
            C Gm[3][3];
            {
                const C irp = fast_rcp(pl[0][wv + 1][lane + 2]), irm = fast_rcp(pl[0][wv + 1][lane]);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    Gm[c][0] = (pl[1 + c][wv + 1][lane + 2] * irp - pl[1 + c][wv + 1][lane] * irm) * scx;
            }
            {
                const C irp = fast_rcp(pl[0][wv + 2][lane + 1]), irm = fast_rcp(pl[0][wv][lane + 1]);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    Gm[c][1] = (pl[1 + c][wv + 2][lane + 1] * irp - pl[1 + c][wv][lane + 1] * irm) * scy;
            }
            {
                const C irp = fast_rcp(qp[0]), irm = fast_rcp(qm[0]);
#pragma unroll
                for (int c = 0; c < 3; ++c) Gm[c][2] = (qp[1 + c] * irp - qm[1 + c] * irm) * scz;
            }
            const C div = Gm[0][0] + Gm[1][1] + Gm[2][2];
            C* tp = T6 + (long long)(k + G) * sz;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = a; b < 3; ++b) {
                    C t = mu * (Gm[a][b] + Gm[b][a]);
                    if (a == b) t += lam * div;
                    *at_plane(tp + (long long)tau_index(a, b) * fs, col) = t;
                }
        }
        __syncthreads();
    }
}

// Stage weight of dt in the output: U1 = Un + dt L, U2 = ... + 1/4 dt L,
// Un+1 = ... + 2/3 dt L (RHS mode: L itself).
template <int MODE>
__device__ __forceinline__ double viscous_weight() {
    return MODE == MODE_STAGE2 ? 0.25 : (MODE == MODE_STAGE3 ? 2.0 / 3.0 : 1.0);
}

// the two sides of the face between cells 2 and 3 of v[0..5]
template <class C, int ORDER>
__device__ __forceinline__ void recon_face(C v0, C v1, C v2, C v3, C v4, C v5, C& l, C& r) {
    if constexpr (ORDER == 5) {
        l = recon_left(v0, v1, v2, v3, v4);
        r = recon_right(v1, v2, v3, v4, v5);
    } else {
        l = recon3_left(v1, v2, v3);
        r = recon3_right(v2, v3, v4);
    }
}

// Viscous flux of the face between cells 2 and 3 of v[f][0..5] (fields
// rho, m_x, m_y, m_z, then tau_xd, tau_yd, tau_zd of the face's direction
// d): per side the momenta's flux is -tau e_d and the energy's
// -(u . tau) e_d with u = m / rho of that side; Fv is the mean of the two
// sides (Fv[0..2] momenta, Fv[3] energy).  The fields go one at a time
// (rho, then each m_c with tau_cd), so that only running sums stay live.
template <class C, int ORDER, class Win>
__device__ __forceinline__ void viscous_face(Win win, C (&Fv)[4]) {
    C v[6];
    win(0, v);
    C rl, rr;
    recon_face<C, ORDER>(v[0], v[1], v[2], v[3], v[4], v[5], rl, rr);
    const C il = fast_rcp(rl), ir = fast_rcp(rr);
    C el = C(0), er = C(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        C ml, mr, tl, tr;
        win(1 + c, v);
        recon_face<C, ORDER>(v[0], v[1], v[2], v[3], v[4], v[5], ml, mr);
        win(4 + c, v);
        recon_face<C, ORDER>(v[0], v[1], v[2], v[3], v[4], v[5], tl, tr);
        Fv[c] = C(-0.5) * (tl + tr);
        el += ml * il * tl;
        er += mr * ir * tr;
    }
    Fv[3] = C(-0.5) * (el + er);
}

constexpr int VISC_TX = 64;
// in-plane fields staged in LDS: rho, m_x, m_y, m_z, tau_xx, tau_xy,
// tau_xz, tau_yy, tau_yz; the x stencil reads fields 0-3 and 4, 5, 6
// (tau_xx, tau_yx, tau_zx), the y stencil 0-3 and 5, 7, 8 (tau_xy,
// tau_yy, tau_zy)
constexpr int VISC_NF = 9;

// F: a storage form (FP64, FP32, 16-bit storage with FP32 arithmetic, or
// the split form; where the stage output is stored in fewer bits than the
// arithmetic, the value the flux kernel rounded is read back, the viscous
// increment added in FP32 and the sum rounded again: in the split form's
// stages 1 and 2 that value is the BF16 difference from U^n).  U (+ D with
// HASD, the split form's later stages): the stage input (ghosts filled);
// T6: its stress (ghosts filled); out: the stage output that the flux
// kernel wrote (or the right-hand side), read and written pointwise.
// speed (last stage, nullable): one CFL maximum per block of the new state
// as stored (cfl_speed in FP64, as the standalone reduction forms it), for
// the next step's dt; a non-physical new state sets *flag.
// Block: 64 x (TY + 1) threads; wave w < TY owns row w of the tile, wave
// TY computes the extra row of y faces and the x faces at the tile's left
// edge.  All faces of one direction run through one instruction sequence.
template <class F, int MODE, int TY, int ORDER, int MINW, bool HASD>
__global__ __launch_bounds__(VISC_TX*(TY + 1), MINW) void k_viscous_tiled(const typename F::TB* __restrict__ U,
                                                                           const typename F::TD* __restrict__ D,
                                                                           const typename F::C* __restrict__ T6,
                                                                           FluxOut<F, MODE>* out,
                                                                           const double* __restrict__ dtp,
                                                                           double dt_fixed, Geom g, int tiles_x,
                                                                           int tiles_y, int zc,
                                                                           double* __restrict__ speed,
                                                                           int* __restrict__ flag) {
    using C = typename F::C;
    using SU = Storage<typename F::TB>;
    using SO = Storage<FluxOut<F, MODE>>;
    static_assert(VISC_TX * (TY + 1) <= 1024, "at most 1024 threads per block");
    constexpr int TX = VISC_TX;
    constexpr int W = TX + 2 * G;
    constexpr int H = TY + 2 * G;
    constexpr int NF = VISC_NF;
    __shared__ C pl[NF][H][W];
    __shared__ C fx[4][TY][TX + 1];
    __shared__ C fy[4][TY + 1][TX];

    const int lane = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.y);
    const int tid = wv * TX + lane;
    int tx, ty, cz;
    tile_coords(xcd_remap(blockIdx.x, gridDim.x), tiles_x, tiles_y, tx, ty, cz);
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = cz * zc;
    const int z1 = min(z0 + zc, nz);
    const long long fs = g.fs;
    const int sy = g.st[1], sz = g.st[2];
    const C ihx = C(g.ih[0]), ihy = C(g.ih[1]), ihz = C(g.ih[2]);
    const C wdt = MODE == MODE_RHS ? C(1) : C(viscous_weight<MODE>() * (dtp ? *dtp : dt_fixed));

    // this thread's column (waves < TY)
    const int i = x0 + lane;
    const int j = y0 + wv;
    const bool own = wv < TY;
    const bool col_load = own && i < nx + G && j < ny + G;
    const bool col_out = own && i < nx && j < ny;
    const uint32_t col = uint32_t((j + G) * sy + (i + G));

    // Field f (0..8 the in-plane fields, 9 tau_zz) at in-plane offset o of
    // a plane: a uniform plane base plus a 32-bit offset per lane
    auto plane_of = [&](auto* a, int f, int plane) {
        plane = __builtin_amdgcn_readfirstlane(plane);
        return a + ((long long)f * fs + (long long)(plane + G) * sz);
    };
    auto ldf = [&](int f, int plane, uint32_t o) -> C {
        if constexpr (!F::SPLIT && std::is_same_v<typename F::TB, C>) {
            // FP64 / FP32: one load through a selected base
            const C* a = f < 4 ? U + (long long)f * fs : T6 + (long long)(f - 4) * fs;
            return SU::load(at_plane(plane_of(a, 0, plane), o));
        } else {
            // 16-bit state, or the split form's U^n (+ difference); FP32 stress
            if (f < 4)
                return F::cvt(F::template load_up<HASD>(plane_of(U, f, plane), HASD ? plane_of(D, f, plane) : nullptr, o));
            return *at_plane(plane_of(T6, f - 4, plane), o);
        }
    };
    // the column's z-stencil fields: rho, m, tau_xz, tau_yz, tau_zz
    auto zfield = [](int f) { return f < 4 ? f : (f == 4 ? 6 : (f == 5 ? 8 : 9)); };
    auto load_col = [&](int plane, C (&v)[7]) {
#pragma unroll
        for (int f = 0; f < 7; ++f) v[f] = ldf(zfield(f), plane, col);
    };

    // register queue: slot p holds plane k-2+p of the seven z fields;
    // columns that are never loaded keep a valid state (their faces are
    // evaluated but discarded)
    C q[7][6];
#pragma unroll
    for (int f = 0; f < 7; ++f)
#pragma unroll
        for (int p = 0; p < 6; ++p) q[f][p] = f == 0 ? C(1) : C(0);
    C nxt[7];
#pragma unroll
    for (int f = 0; f < 7; ++f) nxt[f] = f == 0 ? C(1) : C(0);
    if (col_load) {
#pragma unroll
        for (int p = 0; p < 5; ++p) {
            C v[7];
            load_col(z0 - 3 + p, v);
#pragma unroll
            for (int f = 0; f < 7; ++f) q[f][p + 1] = v[f];
        }
        load_col(z0 + 2, nxt);
    }
    // the column's in-plane stresses that the queue lacks (tau_xx, tau_xy,
    // tau_yy), one plane ahead
    constexpr int PF[3] = {4, 5, 7};
    C pw[3] = {C(0), C(0), C(0)};
    if (col_load) {
#pragma unroll
        for (int e = 0; e < 3; ++e) pw[e] = ldf(PF[e], z0, col);
    }

    // halo of the next plane, prefetched into registers.  The y stencils
    // read rho, m, tau_xy, tau_yy, tau_yz and the x stencils rho, m,
    // tau_xx, tau_xy, tau_xz (seven of the nine fields each), so only
    // those are fetched: the y-halo (2G rows x TX columns x 7 fields) row
    // by row to the waves (lane = column, coalesced), the x-halo (2G
    // columns x TY rows x 7 fields) to the first 7 * 2G * TY threads
    constexpr int NW = TY + 1;
    constexpr int NYR = 7 * 2 * G;
    constexpr int HY = (NYR + NW - 1) / NW;
    constexpr int NXH = 7 * 2 * G * TY;
    static_assert(NXH <= TX * NW, "x halo needs one thread per cell");
    C hy[HY], hx = C(0);
    auto y_slot = [&](int s, int& f, int& cy) -> bool {
        const int rf = wv + s * NW;
        if (rf >= NYR) return false;
        const int q = rf / (2 * G);
        f = q < 4 ? q : (q == 4 ? 5 : (q == 5 ? 7 : 8));
        const int rr = rf - q * 2 * G;
        cy = rr < G ? rr - G : TY + (rr - G);
        const int gy = y0 + cy;
        return i < nx + G && gy >= -G && gy < ny + G;
    };
    auto x_slot = [&](int& f, int& cx, int& cy) -> bool {
        if (tid >= NXH) return false;
        f = tid / (2 * G * TY);
        const int r = tid - f * 2 * G * TY;
        cy = r / (2 * G);
        const int c = r - cy * 2 * G;
        cx = c < G ? c - G : TX + (c - G);
        const int gx = x0 + cx;
        return gx >= -G && gx < nx + G && (y0 + cy) < ny + G;
    };
    auto load_halo = [&](int plane) {
#pragma unroll
        for (int s = 0; s < HY; ++s) {
            int f, cy;
            hy[s] = C(0);
            if (y_slot(s, f, cy)) hy[s] = ldf(f, plane, uint32_t((y0 + cy + G) * sy + (i + G)));
        }
        int f, cx, cy;
        hx = C(0);
        if (x_slot(f, cx, cy)) hx = ldf(f, plane, uint32_t((y0 + cy + G) * sy + (x0 + cx + G)));
    };
    load_halo(z0);

    // last stage: the CFL maximum of this thread's new cells, one LDS slot
    // per thread (the register would stay live across the plane loop)
    constexpr bool FUSE = MODE == MODE_STAGE3;
    __shared__ double smax[FUSE ? VISC_TX * (TY + 1) : 1];
    if (FUSE) smax[tid] = 0.0;
    const bool spd = FUSE && speed != nullptr;
    bool bad = false;

    C Fz_prev[4] = {C(0), C(0), C(0), C(0)};
    for (int k = z0 - 1; k < z1; ++k) {
        // shift the queue; slots hold k-2..k+3 afterwards
#pragma unroll
        for (int f = 0; f < 7; ++f) {
#pragma unroll
            for (int p = 0; p < 5; ++p) q[f][p] = q[f][p + 1];
            q[f][5] = nxt[f];
        }
        if (col_load && k + 1 < z1) load_col(k + 4, nxt);
        C ov[4] = {C(0), C(0), C(0), C(0)};
        C orho = C(1);
        if (k >= z0) {
            // the output's old values, read while the plane is staged (and
            // its density, which these terms leave as it is, for the CFL
            // maximum of the last stage)
            if (col_out) {
#pragma unroll
                for (int f = 0; f < 4; ++f) ov[f] = C(SO::load(at_plane(plane_of(out, 1 + f, k), col)));
                if (spd) orho = C(SO::load(at_plane(plane_of(out, 0, k), col)));
            }
            // A: stage plane k (the tile from the queue and the prefetched
            // in-plane stresses, the halo from the prefetched registers),
            // then prefetch the halo and in-plane stresses of plane k+1
            if (own) {
                pl[0][wv + G][lane + G] = q[0][2];
                pl[1][wv + G][lane + G] = q[1][2];
                pl[2][wv + G][lane + G] = q[2][2];
                pl[3][wv + G][lane + G] = q[3][2];
                pl[4][wv + G][lane + G] = pw[0];
                pl[5][wv + G][lane + G] = pw[1];
                pl[6][wv + G][lane + G] = q[4][2];
                pl[7][wv + G][lane + G] = pw[2];
                pl[8][wv + G][lane + G] = q[5][2];
            }
#pragma unroll
            for (int s = 0; s < HY; ++s) {
                int f, cy;
                if (y_slot(s, f, cy)) pl[f][cy + G][lane + G] = hy[s];
            }
            {
                int f, cx, cy;
                if (x_slot(f, cx, cy)) pl[f][cy + G][cx + G] = hx;
            }
            if (k + 1 < z1) {
                load_halo(k + 1);
                if (col_load) {
#pragma unroll
                    for (int e = 0; e < 3; ++e) pw[e] = ldf(PF[e], k + 1, col);
                }
            }
            __syncthreads();
            // B1: x faces.  Waves < TY: face (x0+lane)+1/2 of row wv; wave
            // TY, lanes < TY: face x0-1/2 of row `lane`.  The face's stencil
            // (cells left-2 .. left+3) sits in LDS columns fi .. fi+5.
            {
                constexpr int XF[7] = {0, 1, 2, 3, 4, 5, 6};
                const int r = own ? wv : lane;
                const int fi = own ? lane + 1 : 0;
                if (own || lane < TY) {
                    C Fv[4];
                    viscous_face<C, ORDER>(
                        [&](int f, C (&v)[6]) {
#pragma unroll
                            for (int c = 0; c < 6; ++c) v[c] = pl[XF[f]][r + G][fi + c];
                        },
                        Fv);
#pragma unroll
                    for (int f = 0; f < 4; ++f) fx[f][r][fi] = Fv[f];
                }
            }
            // B2: y faces.  Waves < TY: face (y0+wv)+1/2 of column lane;
            // wave TY: face y0-1/2.  Stencil rows fj .. fj+5.
            {
                constexpr int YF[7] = {0, 1, 2, 3, 5, 7, 8};
                const int fj = own ? wv + 1 : 0;
                C Fv[4];
                viscous_face<C, ORDER>(
                    [&](int f, C (&v)[6]) {
#pragma unroll
                        for (int c = 0; c < 6; ++c) v[c] = pl[YF[f]][fj + c][lane + G];
                    },
                    Fv);
#pragma unroll
                for (int f = 0; f < 4; ++f) fy[f][fj][lane] = Fv[f];
            }
            __syncthreads();
        }
        // z face k+1/2 from the queue (after the x and y faces: fewer
        // values live across them)
        C Fz[4];
        viscous_face<C, ORDER>(
            [&](int f, C (&v)[6]) {
#pragma unroll
                for (int c = 0; c < 6; ++c) v[c] = q[f][c];
            },
            Fz);
        // C: flux differences (x, y, z) and the stage update
        if (k >= z0 && col_out) {
            C Lv[4] = {C(0), C(0), C(0), C(0)};
#pragma unroll
            for (int f = 0; f < 4; ++f) Lv[f] -= (fx[f][wv][lane + 1] - fx[f][wv][lane]) * ihx;
#pragma unroll
            for (int f = 0; f < 4; ++f) Lv[f] -= (fy[f][wv + 1][lane] - fy[f][wv][lane]) * ihy;
#pragma unroll
            for (int f = 0; f < 4; ++f) Lv[f] -= (Fz[f] - Fz_prev[f]) * ihz;
            double vs[4];
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const C v = ov[f] + wdt * Lv[f];
                SO::store(at_plane(plane_of(out, 1 + f, k), col), v);
                vs[f] = double(SO::stored(v));
            }
            if (spd)
                smax[tid] = fmax(smax[tid], cfl_speed(g, double(orho), vs[0], vs[1], vs[2], vs[3], bad));
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) Fz_prev[f] = Fz[f];
    }
    if (spd) {
        // block maximum: each wave's slots by shuffles, then the waves
        double m = smax[tid];
        for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
        __syncthreads();
        if (lane == 0) smax[wv] = m;
        __syncthreads();
        if (tid == 0) {
            double mm = 0.0;
            for (int w = 0; w <= TY; ++w) mm = fmax(mm, smax[w]);
            speed[blockIdx.x] = mm;
        }
        if (bad) flag[0] = 1;
    }
}

// ---------------------------------------------------------------------------
// Adjoint of the viscous terms (FP64; the right-hand side's part
// L_v(U) = -sum_d (F(+1/2) - F(-1/2)) / h_d of the momenta and energy).
// Reverse order: face fluxes -> reconstructed sides -> cell values of
// rho, m (into the state's cotangent) and of tau (into Tb, 6 components,
// ghost positions included) -> tau's ghost copies folded back -> tau(G)
// -> G by central differences of u = m / rho -> rho, m.
// ---------------------------------------------------------------------------

// Per face l+1/2 (l = -1..n-1) of direction D: the cotangents of the two
// sides' reconstructed rho, m, tau_xD, tau_yD, tau_zD, stored at padded
// position l+1 along D: FV[0..6] left, FV[7..13] right.
template <int D, int ORDER>
__global__ __launch_bounds__(256) void k_adj_visc_face(const double* __restrict__ U, const double* __restrict__ T6,
                                                       const double* __restrict__ Lb, double* __restrict__ FV,
                                                       Geom g) {
    const Line tl = transverse(D);
    const int nd = g.n[D];
    const long long nlines = (long long)g.n[tl.a] * g.n[tl.b];
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nlines * (nd + 1)) return;
    const int f = int(t % (nd + 1));
    const long long line = t / (nd + 1);
    const int ia = int(line % g.n[tl.a]);
    const int ib = int(line / g.n[tl.a]);
    const int sd = g.st[D];
    const long long base = (long long)(ia + G) * g.st[tl.a] + (long long)(ib + G) * g.st[tl.b];
    const int l = f - 1;
    const long long ol = base + (long long)(l + G) * sd;   // left cell of the face
    // face flux cotangents (momenta, energy) from the two cells' L-bar
    double Fb[4];
    for (int c = 0; c < 4; ++c) {
        const double right = (l + 1 <= nd - 1) ? Lb[(1 + c) * g.fs + ol + sd] : 0.0;
        const double left = (l >= 0) ? Lb[(1 + c) * g.fs + ol] : 0.0;
        Fb[c] = (right - left) * g.ih[D];
    }
    // forward: the sides of rho, m, tau_cD from cells l-2..l+3
    double q[7][6];
    for (int p = 0; p < 6; ++p) {
        const long long op = ol + (long long)(p - 2) * sd;
        for (int k = 0; k < 4; ++k) q[k][p] = U[k * g.fs + op];
        for (int c = 0; c < 3; ++c) q[4 + c][p] = T6[(long long)tau_index(c, D) * g.fs + op];
    }
    double rl[7], rr[7];
    for (int k = 0; k < 7; ++k) {
        if constexpr (ORDER == 5) {
            rl[k] = recon_left(q[k][0], q[k][1], q[k][2], q[k][3], q[k][4]);
            rr[k] = recon_right(q[k][1], q[k][2], q[k][3], q[k][4], q[k][5]);
        } else {
            rl[k] = recon3_left(q[k][1], q[k][2], q[k][3]);
            rr[k] = recon3_right(q[k][2], q[k][3], q[k][4]);
        }
    }
    const double il = 1.0 / rl[0], ir = 1.0 / rr[0];
    // reverse of F_c = -1/2 (tl_c + tr_c), F_E = -1/2 sum_c (ml_c il tl_c + mr_c ir tr_c)
    double lb[7] = {0, 0, 0, 0, 0, 0, 0}, rb[7] = {0, 0, 0, 0, 0, 0, 0};
    const double eb = -0.5 * Fb[3];
    double ilb = 0.0, irb = 0.0;
    for (int c = 0; c < 3; ++c) {
        lb[4 + c] += -0.5 * Fb[c] + eb * rl[1 + c] * il;
        rb[4 + c] += -0.5 * Fb[c] + eb * rr[1 + c] * ir;
        lb[1 + c] += eb * il * rl[4 + c];
        rb[1 + c] += eb * ir * rr[4 + c];
        ilb += eb * rl[1 + c] * rl[4 + c];
        irb += eb * rr[1 + c] * rr[4 + c];
    }
    lb[0] -= ilb * il * il;
    rb[0] -= irb * ir * ir;
    const long long of = base + (long long)(f + G) * sd;
    for (int k = 0; k < 7; ++k) {
        FV[k * g.fs + of] = lb[k];
        FV[(7 + k) * g.fs + of] = rb[k];
    }
}

// Transposed reconstruction of the viscous sides: padded cell q along D
// (q = -3..n+2) gathers from the faces whose stencils contain it; rho, m
// add into Ub (the state's padded cotangent), tau_cD into Tb.
template <int D, int ORDER>
__global__ __launch_bounds__(256) void k_adj_visc_gather(const double* __restrict__ FV, double* __restrict__ Ub,
                                                         double* __restrict__ Tb, Geom g) {
    const Line tl = transverse(D);
    const int nd = g.n[D];
    const int np = nd + 2 * G;
    const long long nlines = (long long)g.n[tl.a] * g.n[tl.b];
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nlines * np) return;
    const int qp = int(t % np) - G;
    const long long line = t / np;
    const int ia = int(line % g.n[tl.a]);
    const int ib = int(line / g.n[tl.a]);
    const int sd = g.st[D];
    const long long base = (long long)(ia + G) * g.st[tl.a] + (long long)(ib + G) * g.st[tl.b];
    constexpr int NS = ORDER == 5 ? 5 : 3;
    constexpr int SL = ORDER == 5 ? 2 : 1;
    constexpr int SR = ORDER == 5 ? 1 : 0;
    constexpr double DEN = ORDER == 5 ? 60.0 : 6.0;
    const double CLc[5] = {ORDER == 5 ? 2.0 : -1.0, ORDER == 5 ? -13.0 : 5.0, ORDER == 5 ? 47.0 : 2.0, 27.0, -3.0};
    const double CRc[5] = {ORDER == 5 ? -3.0 : 2.0, ORDER == 5 ? 27.0 : 5.0, ORDER == 5 ? 47.0 : -1.0, -13.0, 2.0};
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int m = 0; m < NS; ++m) {
        const int lL = qp + SL - m;
        if (lL >= -1 && lL <= nd - 1) {
            const long long of = base + (long long)(lL + 1 + G) * sd;
            const double w = CLc[m] / DEN;
            for (int k = 0; k < 7; ++k) acc[k] += w * FV[k * g.fs + of];
        }
        const int lR = qp + SR - m;
        if (lR >= -1 && lR <= nd - 1) {
            const long long of = base + (long long)(lR + 1 + G) * sd;
            const double w = CRc[m] / DEN;
            for (int k = 0; k < 7; ++k) acc[k] += w * FV[(7 + k) * g.fs + of];
        }
    }
    const long long oc = base + (long long)(qp + G) * sd;
    for (int k = 0; k < 4; ++k) Ub[k * g.fs + oc] += acc[k];
    for (int c = 0; c < 3; ++c) Tb[(long long)tau_index(c, D) * g.fs + oc] += acc[4 + c];
}

// tau's cotangent at interior cells (ghost copies folded back, Tf) ->
// the cotangent of G: Gb_ab = mu Tf[ab] for a != b, and
// 2 mu Tf[aa] + lambda sum_c Tf[cc] on the diagonal; written at interior
// cells of Gb (9 fields, row-major a, b; ghosts stay zero).
__global__ __launch_bounds__(256) void k_adj_stress_g(const double* __restrict__ Tf, double* __restrict__ Gb, Geom g,
                                                      double mu, double zeta) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const long long o = cell_offset(g, i, j, k);
    const double lam = zeta - 2.0 * mu / 3.0;
    const double trb = Tf[(long long)tau_index(0, 0) * g.fs + o] + Tf[(long long)tau_index(1, 1) * g.fs + o] +
                       Tf[(long long)tau_index(2, 2) * g.fs + o];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double tb = Tf[(long long)tau_index(a, b) * g.fs + o];
            Gb[(long long)(3 * a + b) * g.fs + o] = a == b ? 2.0 * mu * tb + lam * trb : mu * tb;
        }
}

// G_ab = (u_a(x + e_b) - u_a(x - e_b)) / (2 h_b), u = m / rho: every padded
// cell within one layer of the interior gathers u-bar from the interior
// cells that difference it, then adds rho-bar and m-bar into Ub.
__global__ __launch_bounds__(256) void k_adj_stress_u(const double* __restrict__ U, const double* __restrict__ Gb,
                                                      double* __restrict__ Ub, Geom g) {
    const int i = int(blockIdx.x * blockDim.x + threadIdx.x) - 1;
    const int j = int(blockIdx.y * blockDim.y + threadIdx.y) - 1;
    const int k = int(blockIdx.z) - 1;
    if (i > g.n[0] || j > g.n[1] || k > g.n[2]) return;
    const int idx[3] = {i, j, k};
    // a cell outside the interior in two axes (an edge or corner of the
    // ghost layer, never filled) is differenced by no interior cell
    int outside = 0;
    for (int d = 0; d < 3; ++d) outside += (idx[d] < 0 || idx[d] >= g.n[d]) ? 1 : 0;
    if (outside > 1) return;
    const long long o = cell_offset(g, i, j, k);
    double ub[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < 3; ++b) {
        const double sc = 0.5 * g.ih[b];
        // the interior neighbours x = q - e_b (which reads q as its + side)
        // and x = q + e_b (which reads q as its - side)
        const bool hm = idx[b] - 1 >= 0 && idx[b] - 1 < g.n[b];
        const bool hp = idx[b] + 1 >= 0 && idx[b] + 1 < g.n[b];
        for (int a = 0; a < 3; ++a) {
            const double* Ga = Gb + (long long)(3 * a + b) * g.fs;
            if (hm) ub[a] += sc * Ga[o - g.st[b]];
            if (hp) ub[a] -= sc * Ga[o + g.st[b]];
        }
    }
    const double rho = U[o];
    const double r = 1.0 / rho;
    double rb = 0.0;
    for (int a = 0; a < 3; ++a) {
        Ub[(long long)(1 + a) * g.fs + o] += ub[a] * r;
        rb -= ub[a] * U[(long long)(1 + a) * g.fs + o] * r * r;
    }
    Ub[o] += rb;
}

}  // namespace igr
