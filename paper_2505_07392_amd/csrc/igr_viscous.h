// Viscous terms of the Navier-Stokes balances, eqs. (2)-(3), with the
// stress of eq. (5): tau = mu (G + G^T) + (zeta - 2 mu / 3) tr(G) I,
// G_ij = d u_i / d x_j.  They are added to a right-hand side or RK stage
// that the inviscid flux kernel has already written ("sequential summation
// of right-hand side contributions"):
//
//   k_vel_grad   G at interior cells by second-order central differences of
//                u = m / rho (the paper: second-order derivatives of u
//                suffice); ghost cells of G follow Sigma's rule (k_bc_sigma
//                per component);
//   k_viscous    per cell and direction d, the viscous flux at both faces:
//                each side's tau e_d reconstructed from the cell-centre
//                stresses with the weights of the conserved variables
//                (Algorithm 1 reconstructs the gradients with the same
//                coefficients; tau is linear in G), each side's velocity
//                from the reconstructed conserved variables, and the mean
//                of the two sides' fluxes -tau e_d (momenta) and
//                -(u . tau) e_d (energy); the divergence is scaled by the
//                stage's weight of dt and added to the output.
#pragma once

#include "igr_flux.h"

namespace igr {

template <class F, bool HASD>
__global__ __launch_bounds__(256) void k_vel_grad(const typename F::TB* __restrict__ U,
                                                  const typename F::TD* __restrict__ D,
                                                  typename F::C* __restrict__ Gout, Geom g) {
    using C = typename F::C;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const long long o = cell_offset(g, i, j, k);
    const long long fs = g.fs;
    auto get = [&](long long off) { return F::cvt(F::template load_u<HASD>(U, D, off)); };
    for (int d = 0; d < 3; ++d) {
        const long long op = o + g.st[d], om = o - g.st[d];
        const C irp = C(1) / get(op), irm = C(1) / get(om);
        const C sc = C(0.5) * C(g.ih[d]);
        for (int c = 0; c < 3; ++c)
            Gout[(3 * c + d) * fs + o] = (get((1 + c) * fs + op) * irp - get((1 + c) * fs + om) * irm) * sc;
    }
}

// Stage weight of dt in the output: U1 = Un + dt L, U2 = ... + 1/4 dt L,
// Un+1 = ... + 2/3 dt L (RHS mode: L itself).
template <int MODE>
__device__ __forceinline__ double viscous_weight() {
    return MODE == MODE_STAGE2 ? 0.25 : (MODE == MODE_STAGE3 ? 2.0 / 3.0 : 1.0);
}

template <class F, int MODE, int ORDER, bool HASD>
__global__ __launch_bounds__(256) void k_viscous(const typename F::TB* __restrict__ U,
                                                 const typename F::TD* __restrict__ D,
                                                 const typename F::C* __restrict__ Gp, FluxOut<F, MODE>* out,
                                                 const double* __restrict__ dtp, double dt_fixed, Geom g,
                                                 double mu_, double zeta_) {
    using C = typename F::C;
    using SO = Storage<FluxOut<F, MODE>>;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const long long o = cell_offset(g, i, j, k);
    const long long fs = g.fs;
    const C mu = C(mu_), lam = C(zeta_) - C(2) * C(mu_) / C(3);
    auto get = [&](long long off) { return F::cvt(F::template load_u<HASD>(U, D, off)); };
    auto gr = [&](int a, int b, long long off) { return Gp[(3 * a + b) * fs + off]; };   // d u_a / d x_b
    C Lv[4] = {C(0), C(0), C(0), C(0)};   // momenta, energy
    for (int d = 0; d < 3; ++d) {
        // cells i-3 .. i+3 along d: conserved (rho, m) and the stress column tau_kd
        C v[7][4], t[7][3];
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            const long long oq = o + (long long)(q - 3) * g.st[d];
#pragma unroll
            for (int f = 0; f < 4; ++f) v[q][f] = get(f * fs + oq);
            const C div = gr(0, 0, oq) + gr(1, 1, oq) + gr(2, 2, oq);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                C tk = mu * (gr(c, d, oq) + gr(d, c, oq));
                if (c == d) tk += lam * div;
                t[q][c] = tk;
            }
        }
        // faces i-1/2 (s = 0: cells q = 0..5) and i+1/2 (s = 1: q = 1..6)
        C Fm[2][3], Fe[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            C rL[4], rR[4], tL[3], tR[3];
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                if constexpr (ORDER == 5) {
                    rL[f] = recon_left(v[s][f], v[s + 1][f], v[s + 2][f], v[s + 3][f], v[s + 4][f]);
                    rR[f] = recon_right(v[s + 1][f], v[s + 2][f], v[s + 3][f], v[s + 4][f], v[s + 5][f]);
                } else {
                    rL[f] = recon3_left(v[s + 1][f], v[s + 2][f], v[s + 3][f]);
                    rR[f] = recon3_right(v[s + 2][f], v[s + 3][f], v[s + 4][f]);
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if constexpr (ORDER == 5) {
                    tL[c] = recon_left(t[s][c], t[s + 1][c], t[s + 2][c], t[s + 3][c], t[s + 4][c]);
                    tR[c] = recon_right(t[s + 1][c], t[s + 2][c], t[s + 3][c], t[s + 4][c], t[s + 5][c]);
                } else {
                    tL[c] = recon3_left(t[s + 1][c], t[s + 2][c], t[s + 3][c]);
                    tR[c] = recon3_right(t[s + 2][c], t[s + 3][c], t[s + 4][c]);
                }
            }
            const C iL = C(1) / rL[0], iR = C(1) / rR[0];
            C eL = C(0), eR = C(0);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Fm[s][c] = C(-0.5) * (tL[c] + tR[c]);
                eL += rL[1 + c] * iL * tL[c];
                eR += rR[1 + c] * iR * tR[c];
            }
            Fe[s] = C(-0.5) * (eL + eR);
        }
        const C ih = C(g.ih[d]);
#pragma unroll
        for (int c = 0; c < 3; ++c) Lv[c] -= (Fm[1][c] - Fm[0][c]) * ih;
        Lv[3] -= (Fe[1] - Fe[0]) * ih;
    }
    const C w = MODE == MODE_RHS ? C(1) : C(viscous_weight<MODE>() * (dtp ? *dtp : dt_fixed));
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const long long of = (1 + f) * fs + o;
        SO::store(out + of, SO::load(out + of) + w * Lv[f]);
    }
}

}  // namespace igr
