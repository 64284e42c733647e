"""Pins of the oracle's inflow ghosts on the x-min face (paper, "Example
simulation result": engines enter as inflow boundary conditions; eq. (4),
the ideal-gas law, turns the primitive jet state into conserved variables).

The ghost state is rebuilt here column by column with plain Python loops
and floats, independently of ``patch_weights``, ``jet_conserved`` and
``pad_state``:

* the owner of a column is the disc whose centre is nearest to the column's
  cell centre ((j+1/2) dy, (k+1/2) dz), found by an explicit loop that keeps
  the lowest index on ties;
* the blend weight is chi = (1 - tanh((s - r) / w)) / 2 at distance s for
  an edge width w > 0, and the indicator s <= r (inclusive) for w = 0;
* the jet's conserved state is (rho, rho u, rho v, rho w,
  p / (gamma - 1) + rho |u|^2 / 2);
* every one of the three ghost layers holds chi U_jet + (1 - chi) U_0 with
  U_0 the column's first interior cell.

The geometry uses spacings that are powers of two, so that a column centre
equidistant from two disc centres is an exact tie and a column on a disc's
rim sits exactly at s = r; a wrong tie rule, an exclusive rim or a wrong
blend radius then changes values, not just rounding.
"""

import math

import pytest
import torch

from oracle import igr_ref as ref

GAMMA = 1.4
H = 0.25                       # dx = dy = dz (exact in binary)
NX, NY, NZ = 4, 8, 6


def _discs(width):
    # centres (yc, zc), radius, primitive state (rho, ux, uy, uz, p)
    return [
        # A and B are mirror images about y = 0.625 (column j = 2): every
        # column with y = 0.625 is equidistant from both (an exact tie)
        ref.Patch(yc=0.375, zc=0.625, r=0.25, rho=0.5, ux=3.0, uy=0.25, uz=-0.5, p=8.0, width=width),
        ref.Patch(yc=0.875, zc=0.625, r=0.30, rho=0.8, ux=-1.0, uy=0.0, uz=0.75, p=2.0, width=width),
        # C overlaps the face edge z = 0 (its disc extends past the domain)
        ref.Patch(yc=1.625, zc=0.0625, r=0.40, rho=1.7, ux=0.5, uy=-2.0, uz=1.0, p=0.6, width=width),
    ]


def _problem(width, faces=None):
    faces = faces or (ref.EXTRAP, ref.EXTRAP, ref.PERIODIC, ref.PERIODIC, ref.EXTRAP, ref.EXTRAP)
    return ref.Problem(NX, NY, NZ, H, H, H, gamma=GAMMA, alpha=0.0, faces=faces, patches=tuple(_discs(width)))


def _state(seed=3):
    g = torch.Generator().manual_seed(seed)
    rho = 0.5 + torch.rand((NZ, NY, NX), generator=g, dtype=torch.float64)
    m = torch.rand((3, NZ, NY, NX), generator=g, dtype=torch.float64) - 0.5
    E = 3.0 + torch.rand((NZ, NY, NX), generator=g, dtype=torch.float64)
    return torch.cat([rho[None], m, E[None]])


def _brute_ghost(discs, U, j, k):
    """Expected x-min ghost (5 values) of column (j, k), and its owner/chi."""
    y = (j + 0.5) * H
    z = (k + 0.5) * H
    owner, best = -1, math.inf
    for q, d in enumerate(discs):
        d2 = (y - d.yc) ** 2 + (z - d.zc) ** 2
        if d2 < best:             # strict: the lowest index keeps a tie
            owner, best = q, d2
    d = discs[owner]
    s = math.sqrt(best)
    if d.width > 0:
        chi = 0.5 * (1.0 - math.tanh((s - d.r) / d.width))
    else:
        chi = 1.0 if s <= d.r else 0.0
    ke = 0.5 * d.rho * (d.ux * d.ux + d.uy * d.uy + d.uz * d.uz)
    jet = [d.rho, d.rho * d.ux, d.rho * d.uy, d.rho * d.uz, d.p / (GAMMA - 1.0) + ke]
    first = [float(U[f, k, j, 0]) for f in range(5)]
    ghost = [chi * jet[f] + (1.0 - chi) * first[f] for f in range(5)]
    return ghost, owner, chi


@pytest.mark.parametrize("width", [0.0, 0.15])
def test_inflow_ghosts_brute_force(width):
    prob = _problem(width)
    U = _state()
    V = ref.pad_state(prob, U)
    G = ref.G
    discs = _discs(width)
    ties = rims = 0
    for k in range(NZ):
        for j in range(NY):
            exp, owner, chi = _brute_ghost(discs, U, j, k)
            y = (j + 0.5) * H
            if y == 0.625 and owner == 0:
                ties += 1
            if width == 0 and chi == 1.0 and (y - discs[owner].yc) ** 2 + ((k + 0.5) * H - discs[owner].zc) ** 2 \
                    == discs[owner].r ** 2:
                rims += 1
            for layer in range(G):
                got = V[:, k + G, j + G, layer]
                for f in range(5):
                    e = exp[f]
                    assert abs(float(got[f]) - e) <= 1e-15 * max(1.0, abs(e)), (width, j, k, layer, f)
    assert ties == NZ           # the tie column exists in every z row
    if width == 0:
        assert rims >= 1        # a column sits exactly on a rim (inclusive)


def test_inflow_owner_and_chi_tables():
    # the oracle's owner/chi tables against the brute force (both widths)
    U = _state()
    for width in (0.0, 0.15):
        prob = _problem(width)
        owner, chi = ref.patch_weights(prob)
        for k in range(NZ):
            for j in range(NY):
                _, o, c = _brute_ghost(_discs(width), U, j, k)
                assert int(owner[k, j]) == o
                assert abs(float(chi[k, j]) - c) <= 1e-15


def test_inflow_other_faces_untouched_and_tensor_jets():
    # the x-max face stays a zero-gradient copy; tensor-valued jet
    # parameters (the differentiable path) give the same ghosts
    prob = _problem(0.15)
    U = _state(seed=5)
    V = ref.pad_state(prob, U)
    G = ref.G
    for layer in range(G):
        assert torch.equal(V[:, G:-G, G:-G, NX + G + layer], U[:, :, :, NX - 1])
    tp = tuple(ref.Patch(d.yc, d.zc, d.r, torch.tensor(d.rho, dtype=torch.float64),
                         torch.tensor(d.ux, dtype=torch.float64), torch.tensor(d.uy, dtype=torch.float64),
                         torch.tensor(d.uz, dtype=torch.float64), torch.tensor(d.p, dtype=torch.float64),
                         d.width) for d in prob.patches)
    prob_t = ref.Problem(NX, NY, NZ, H, H, H, gamma=GAMMA, faces=prob.faces, patches=tp)
    assert torch.equal(ref.pad_state(prob_t, U), V)


def test_inflow_mistakes_are_caught():
    # plausible mistakes in the ghost assembly change values the brute force
    # pins: the highest index on ties, an exclusive rim, and the blend taken
    # about the diameter instead of the radius
    U = _state()
    discs = _discs(0.0)
    j, k = 2, 2                                    # the tie column
    exp, owner, _ = _brute_ghost(discs, U, j, k)
    assert owner == 0
    alt = list(discs)
    alt[0], alt[1] = discs[1], discs[0]            # swapping the order flips the owner
    exp_alt, _, _ = _brute_ghost(alt, U, j, k)
    assert max(abs(a - b) for a, b in zip(exp, exp_alt)) > 1e-3
    # a column exactly on disc 0's rim: inclusive gives chi = 1
    y, z = 0.375, 0.875                            # j = 1, k = 3: s = 0.25 = r
    assert (y - discs[0].yc) ** 2 + (z - discs[0].zc) ** 2 == discs[0].r ** 2
    _, o, c = _brute_ghost(discs, U, 1, 3)
    assert o == 0 and c == 1.0
    # width > 0: chi is 1/2 exactly at s = r and depends on r, not 2r
    d = ref.Patch(yc=0.625, zc=0.375, r=0.25, rho=1.0, ux=0.0, uy=0.0, uz=0.0, p=1.0, width=0.1)
    prob = ref.Problem(NX, NY, NZ, H, H, H, gamma=GAMMA, faces=_problem(0.0).faces, patches=(d,))
    _, chi = ref.patch_weights(prob)
    # column (j=1, k=1): centre (0.375, 0.375), s = 0.25 = r
    assert abs(float(chi[1, 1]) - 0.5) <= 1e-15
