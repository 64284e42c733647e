// Tiled, z-marching fused flux kernel.
//
// One block owns a 64 x TY column tile of the x-y plane and marches through
// a chunk of z planes.  For each plane k:
//   A  the plane (six fields rho, m, E, Sigma, with a three-cell x/y halo;
//      two for third order) is staged in LDS: interior cells from the
//      register queue of each thread's column, halo cells from global memory;
//   B  every face is computed once: x faces (i+1/2) and y faces (j-1/2)
//      from the LDS plane, the z face (k+1/2) from the column's register
//      queue of planes k-2..k+3; x/y face fluxes go to LDS;
//   C  each cell takes the flux differences, forms L(U) and the SSP-RK3
//      stage combination, and stores the result.
// The block has TY+1 waves: wave w < TY owns row w of the tile; wave TY
// computes the extra row of y faces and the x faces at the tile's left
// edge.  All faces of one direction run through one instruction sequence,
// so equal inputs give bitwise equal fluxes (a uniform state stays exactly
// uniform, transverse momentum of a planar problem stays exactly zero).
#pragma once

#include "igr_kernels.h"

namespace igr {

constexpr int FLUX_TX = 64;

// LLF flux at the face between cells 2 and 3 of v[field][0..5] (cells
// i-2..i+3 around face i+1/2) with ORDER-th order reconstruction (5 or 3;
// the third-order stencils use cells i-1..i+2 only).
template <class C, int ORDER>
__device__ __forceinline__ void face_flux6(const C (&v)[6][6], int d, C gamma, C F[5], bool& bad) {
    C Q[6][2];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        if constexpr (ORDER == 5) {
            Q[f][0] = recon_left(v[f][0], v[f][1], v[f][2], v[f][3], v[f][4]);
            Q[f][1] = recon_right(v[f][1], v[f][2], v[f][3], v[f][4], v[f][5]);
        } else {
            Q[f][0] = recon3_left(v[f][1], v[f][2], v[f][3]);
            Q[f][1] = recon3_right(v[f][2], v[f][3], v[f][4]);
        }
    }
    C UL[5], UR[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        UL[f] = Q[f][0];
        UR[f] = Q[f][1];
    }
    llf_flux<C>(UL, UR, Q[5][0], Q[5][1], d, gamma, F, bad);
}

// Element type of a stage's output: the state's type, except the stage
// buffers of the split form (the bfloat16 differences from U^n).
template <class F, int MODE>
using FluxOut = std::conditional_t<F::SPLIT && (MODE == MODE_STAGE1 || MODE == MODE_STAGE2), typename F::TD,
                                   typename F::TB>;

// F: storage form (Plain<T> or Split).  The stage input is U (+ D with
// HASD, the split form's stage difference); Un is U^n for the pointwise
// reads of stages 2 and 3 of the plain forms (the split form reads U and D
// there).  Split outputs: stage 1 and 2 write the difference of the next
// stage state from U^n, stage 3 writes U^(n+1) (FP32, not in place: the
// stencil still reads U^n).
template <class F, int MODE, int TY, int ORDER, bool HASD = false>
__global__ __launch_bounds__(FLUX_TX*(TY + 1)) void k_flux_tiled(
    const typename F::TB* __restrict__ U, const typename F::TD* __restrict__ D,
    const typename F::TS* __restrict__ Sg, const typename F::TB* Un, FluxOut<F, MODE>* out,
    const double* __restrict__ dtp, double dt_fixed, Geom g, int* __restrict__ flag, int tiles_x, int tiles_y,
    int zc, double* __restrict__ speed, typename F::TS* __restrict__ sig_out) {
    using C = typename F::C;
    using RU = typename F::RU;
    using SO = Storage<FluxOut<F, MODE>>;
    using SS = Storage<typename F::TS>;
    constexpr int TX = FLUX_TX;
    // LDS halo width: the reconstruction's reach (three cells, two for
    // third order; the arrays keep G ghost layers either way).  A face's
    // six-cell window v[0..5] (cells -3..+2 around it) is read from LDS
    // for the slots the reconstruction uses, PO..5-PO.
    constexpr int HG = ORDER == 5 ? G : 2;
    constexpr int PO = G - HG;
    constexpr int W = TX + 2 * HG;
    constexpr int H = TY + 2 * HG;
    __shared__ C pl[6][H][W];
    __shared__ C fx[5][TY][TX + 1];
    __shared__ C fy[5][TY + 1][TX];

    const int lane = threadIdx.x;
    // the wave index is uniform in the wave (blocks are 64 wide): SGPR
    // arithmetic for everything that depends on the row only
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
    const C gamma = C(g.gamma);
    // face fluxes come from llf_flux scaled by 1/LLF_SCALE
    const C ihx = LLF_SCALE<C> * C(g.ih[0]), ihy = LLF_SCALE<C> * C(g.ih[1]), ihz = LLF_SCALE<C> * C(g.ih[2]);
    const C dt = C(dtp ? *dtp : dt_fixed);

    // this thread's column (waves < TY): loads padded cells that exist
    const int i = x0 + lane;
    const int j = y0 + wv;
    const bool own = wv < TY;
    const bool col_load = own && i < nx + G && j < ny + G;
    const bool col_out = own && i < nx && j < ny;
    const long long col = (long long)(j + G) * sy + (i + G);
    const uint32_t col32 = uint32_t(col);   // in-plane offset (at_plane)
    // base of field f of array a at a plane: uniform
    // element offset of a plane.  In the FP32-arithmetic kernels without a
    // stage difference the plane index goes through readfirstlane (it is
    // uniform), so that the 64-bit product stays on the scalar unit; the
    // FP64 and difference kernels keep it in a vector register (on the
    // scalar unit their scalar registers overflow and spill)
    constexpr bool ZUNI = sizeof(C) == 4 && !HASD;
    auto zoff = [&](int plane) {
        if constexpr (ZUNI) plane = __builtin_amdgcn_readfirstlane(plane);
        return (long long)(plane + G) * sz;
    };
    auto fplane = [&](auto* a, int f, int plane) { return a + ((long long)f * fs + zoff(plane)); };

    // register queue: planes k-2 .. k+3 of the six fields (index 0..5)
    C q[6][6];
    C Fz_prev[5];
    bool bad = false;
    // fused CFL maximum of the last stage: one LDS slot per thread, since a
    // register carried through the plane loop would raise its peak (FP64
    // stage 3: 251 VGPRs, no spill)
    constexpr bool FUSE = MODE == MODE_STAGE3;
    __shared__ double smax[FUSE ? FLUX_TX * (TY + 1) : 1];
    if (FUSE) smax[tid] = 0.0;
    // columns that are never loaded keep a valid state (their faces are
    // evaluated but discarded)
#pragma unroll
    for (int f = 0; f < 6; ++f)
#pragma unroll
        for (int p = 0; p < 6; ++p) q[f][p] = f == 0 ? C(1) : (f == 4 ? C(2.5) : C(0));
#pragma unroll
    for (int f = 0; f < 5; ++f) Fz_prev[f] = C(0);

    // prefetched values stay in the storage's register form RU until used
    // (a 16-bit value converted at its load would wait for that load)
    // Plane base + 32-bit offset addressing, except for the split form's
    // later stages, whose base + difference loads it leaves with more live
    // registers (spills)
    constexpr bool PLANE_ADDR = !HASD;
    auto load_col = [&](int plane, RU (&v)[6]) {
        if constexpr (PLANE_ADDR) {
#pragma unroll
            for (int f = 0; f < 5; ++f) v[f] = F::template load_up<false>(fplane(U, f, plane), nullptr, col32);
            v[5] = F::load_sp(fplane(Sg, 0, plane), col32);
        } else {
            const long long o = col + zoff(plane);
#pragma unroll
            for (int f = 0; f < 5; ++f) v[f] = F::template load_u<HASD>(U, D, f * fs + o);
            v[5] = F::load_s(Sg, o);
        }
    };
    // prime with planes z0-3 .. z0+1 (slot p holds plane z0-3+p) and keep
    // plane z0+2 in `nxt`; every iteration shifts, moves `nxt` into slot 5
    // and issues the load of the plane after it, so each column load has a
    // whole iteration to arrive.  The loop starts at k = z0 - 1 to compute
    // face z0 - 1/2 with the same code as every other z face.
    RU nxt[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) nxt[f] = RU{};
    if (col_load) {
#pragma unroll
        for (int p = 0; p < 5; ++p) {
            RU v[6];
            load_col(z0 - 3 + p, v);
#pragma unroll
            for (int f = 0; f < 6; ++f) q[f][p + 1] = F::cvt(v[f]);
        }
        load_col(z0 + 2, nxt);
    }

    // halo of the next plane, prefetched into registers.  Regular pattern:
    // the y-halo (2 HG rows x TX columns x 6 fields) goes row by row to the
    // waves (lane = column, coalesced); the x-halo (2 HG columns x TY rows x
    // 6 fields) to the first 6 * 2 HG * TY threads.
    constexpr int NW = TY + 1;                   // waves per block
    constexpr int NYR = 6 * 2 * HG;              // y-halo rows over all fields
    constexpr int HY = (NYR + NW - 1) / NW;      // y-halo rows per wave
    constexpr int NXH = 6 * 2 * HG * TY;         // x-halo cells over all fields
    RU hy[HY], hx = RU{};
    auto y_slot = [&](int s, int& f, int& cy) -> bool {
        const int rf = wv + s * NW;
        if (rf >= NYR) return false;
        f = rf / (2 * HG);
        const int rr = rf - f * 2 * HG;
        cy = rr < HG ? rr - HG : TY + (rr - HG);
        const int gy = y0 + cy;
        return (x0 + lane) < nx + G && gy >= -G && gy < ny + G;
    };
    auto x_slot = [&](int& f, int& cx, int& cy) -> bool {
        if (tid >= NXH) return false;
        f = tid / (2 * HG * TY);
        const int r = tid - f * 2 * HG * TY;
        cy = r / (2 * HG);
        const int c = r - cy * 2 * HG;
        cx = c < HG ? c - HG : TX + (c - HG);
        const int gx = x0 + cx;
        return gx >= -G && gx < nx + G && (y0 + cy) < ny + G;
    };
    auto load_halo = [&](int plane) {
        const long long zo = zoff(plane);
#pragma unroll
        for (int s = 0; s < HY; ++s) {
            int f, cy;
            hy[s] = RU{};
            // the field of a y-halo row is uniform in the wave
            if (y_slot(s, f, cy)) {
                if constexpr (PLANE_ADDR) {
                    const uint32_t o = uint32_t((y0 + cy + G) * sy + (x0 + lane + G));
                    if (f == 5)
                        hy[s] = F::load_sp(fplane(Sg, 0, plane), o);
                    else
                        hy[s] = F::template load_up<false>(fplane(U, f, plane), nullptr, o);
                } else {
                    hy[s] = F::template load_field<HASD>(U, D, Sg, f, fs,
                                                         zo + (long long)(y0 + cy + G) * sy + (x0 + lane + G));
                }
            }
        }
        int f, cx, cy;
        hx = RU{};
        if (x_slot(f, cx, cy))
            hx = F::template load_field<HASD>(U, D, Sg, f, fs, zo + (long long)(y0 + cy + G) * sy + (x0 + cx + G));
    };
    load_halo(z0);

    // pointwise values of stages 2 and 3: plain forms U^n (unv); split form
    // the stage's difference from U^n (und)
    C unv[5], und[5];
    RU un_next[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        unv[f] = C(0);
        und[f] = C(0);
        un_next[f] = RU{};
    }
    for (int k = z0 - 1; k < z1; ++k) {
        // shift the queue; slots hold k-2..k+3 afterwards
#pragma unroll
        for (int f = 0; f < 6; ++f) {
#pragma unroll
            for (int p = 0; p < 5; ++p) q[f][p] = q[f][p + 1];
            if (col_load) q[f][5] = F::cvt(nxt[f]);
        }
        if (col_load && k + 1 < z1) load_col(k + 4, nxt);
        // Un (read pointwise by stages 2 and 3) is fetched one plane ahead
        if (MODE == MODE_STAGE2 || MODE == MODE_STAGE3) {
#pragma unroll
            for (int f = 0; f < 5; ++f) {
                if constexpr (F::SPLIT)
                    und[f] = F::cvt(RU{0.0f, un_next[f].d});
                else
                    unv[f] = F::cvt(un_next[f]);
            }
            if (col_out && k + 1 < z1) {
#pragma unroll
                for (int f = 0; f < 5; ++f) {
                    if constexpr (F::SPLIT)
                        un_next[f].d = D[f * fs + col + zoff(k + 1)].bits;
                    else
                        un_next[f] = F::template load_up<false>(fplane(Un, f, k + 1), nullptr, col32);
                }
            }
        }
        const bool body = k >= z0;
        if (body) {
            // A: stage plane k in LDS (interior from the queue, halo from the
            // prefetched registers), then prefetch the halo of plane k+1
            if (own) {
#pragma unroll
                for (int f = 0; f < 6; ++f) pl[f][wv + HG][lane + HG] = q[f][2];
            }
#pragma unroll
            for (int s = 0; s < HY; ++s) {
                int f, cy;
                if (y_slot(s, f, cy)) pl[f][cy + HG][lane + HG] = F::cvt(hy[s]);
            }
            {
                int f, cx, cy;
                if (x_slot(f, cx, cy)) pl[f][cy + HG][cx + HG] = F::cvt(hx);
            }
            if (k + 1 < z1) load_halo(k + 1);
            __syncthreads();
            {
                // faces one direction at a time (the register budget sets
                // the tile height, and more waves beat more independent
                // chains per wave)
                // B1: x faces.  Waves < TY: face (x0+lane)+1/2 of row wv;
                // wave TY, lanes < TY: face x0-1/2 of row `lane`.  One code path.
                {
                    const int r = own ? wv : lane;
                    const int fi = own ? lane + 1 : 0;       // face index: face (x0 + fi - 1/2)
                    const int gxf = x0 + fi - 1;             // cell left of the face
                    const bool act = (own || lane < TY) && (y0 + r) < ny && gxf >= -1 && gxf < nx;
                    if (act) {
                        C v[6][6];
#pragma unroll
                        for (int f = 0; f < 6; ++f)
#pragma unroll
                            for (int p = 0; p < 6; ++p)
                                v[f][p] = (p >= PO && p < 6 - PO) ? pl[f][r + HG][fi + p - PO] : C(0);
                        C Fl[5];
                        face_flux6<C, ORDER>(v, 0, gamma, Fl, bad);
#pragma unroll
                        for (int f = 0; f < 5; ++f) fx[f][r][fi] = Fl[f];
                    }
                }
                // B2: y faces (y0+wv)-1/2 for wv = 0..TY, column lane
                {
                    const int gyf = y0 + wv;                 // cell above the face
                    const bool act = (x0 + lane) < nx && gyf >= 0 && gyf <= ny;
                    if (act) {
                        C v[6][6];
#pragma unroll
                        for (int f = 0; f < 6; ++f)
#pragma unroll
                            for (int p = 0; p < 6; ++p)
                                v[f][p] = (p >= PO && p < 6 - PO) ? pl[f][wv + p - PO][lane + HG] : C(0);
                        C Fl[5];
                        face_flux6<C, ORDER>(v, 1, gamma, Fl, bad);
#pragma unroll
                        for (int f = 0; f < 5; ++f) fy[f][wv][lane] = Fl[f];
                    }
                }
            }
        }
        // B3: z face k+1/2 from the queue (also at k = z0-1 to prime Fz_prev)
        C Fz[5];
        if (col_out) {
            C v[6][6];
#pragma unroll
            for (int f = 0; f < 6; ++f)
#pragma unroll
                for (int p = 0; p < 6; ++p) v[f][p] = q[f][p];
            face_flux6<C, ORDER>(v, 2, gamma, Fz, bad);
        }
        if (body) {
            __syncthreads();
            // C: divergence and stage update
            if (col_out) {
                double vs[5];
                C L[5];
#pragma unroll
                for (int f = 0; f < 5; ++f) {
                    C l = C(0);
                    l -= (fx[f][wv][lane + 1] - fx[f][wv][lane]) * ihx;
                    l -= (fy[f][wv + 1][lane] - fy[f][wv][lane]) * ihy;
                    l -= (Fz[f] - Fz_prev[f]) * ihz;
                    L[f] = l;
                }
#pragma unroll
                for (int f = 0; f < 5; ++f) {
                    C v;
                    if (MODE == MODE_RHS) {
                        v = L[f];
                    } else if constexpr (F::SPLIT) {
                        // differences from U^n: U1 - Un = dt L(Un);
                        // U2 - Un = 1/4 ((U1 - Un) + dt L(U1)); and
                        // Un+1 = Un + 2/3 ((U2 - Un) + dt L(U2))
                        //      = U2 + 2/3 dt L(U2) - 1/3 (U2 - Un)
                        // with U2 the stencil's centre value (Un + delta in FP32)
                        if (MODE == MODE_STAGE1)
                            v = dt * L[f];
                        else if (MODE == MODE_STAGE2)
                            v = C(0.25) * (und[f] + dt * L[f]);
                        else
                            v = q[f][2] + ((C(2) / C(3)) * (dt * L[f]) - (C(1) / C(3)) * und[f]);
                    } else if (MODE == MODE_STAGE1) {
                        v = q[f][2] + dt * L[f];
                    } else if (MODE == MODE_STAGE2) {
                        v = C(0.75) * unv[f] + C(0.25) * (q[f][2] + dt * L[f]);
                    } else {
                        v = unv[f] * (C(1) / C(3)) + (C(2) / C(3)) * (q[f][2] + dt * L[f]);
                    }
                    SO::store(at_plane(fplane(out, f, k), col32), v);
                    if (FUSE) vs[f] = double(SO::stored(v));
                }
                // last stage: the solved Sigma of this plane into the caller's
                // buffer when the solve ended in the scratch copy
                if (MODE == MODE_STAGE3 && sig_out != nullptr) SS::store(at_plane(fplane(sig_out, 0, k), col32), q[5][2]);
                // last stage: CFL speed of the new state as stored (for the
                // next step's dt), when the caller asked for it
                if (FUSE && speed != nullptr)
                    smax[tid] = fmax(smax[tid], cfl_speed(g, vs[0], vs[1], vs[2], vs[3], vs[4], bad));
            }
        }
        if (col_out) {
#pragma unroll
            for (int f = 0; f < 5; ++f) Fz_prev[f] = Fz[f];
        }
        // the next iteration overwrites pl only after every wave passed the
        // second barrier above, and fx/fy only after its first barrier
    }
    if (FUSE && speed != nullptr) {
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
    }
    if (bad) flag[0] = 1;
}

}  // namespace igr
