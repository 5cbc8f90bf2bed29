"""The single-mode tile cycle (k_cycle1_down / k_cycle1_up) computes on each
tile exactly what the whole-grid steps compute on the tile's core.

The tile sizes and halos are read from the HIP source; this CPU emulation
replays the kernels' thread-to-node mapping, colour passes, residual,
restriction, prolongation and output ownership on random stencils and checks
(a) every output node is written once and (b) the values equal the same
operations applied to the whole grid, to the last bit (float64).  A halo one
node too thin in either direction makes (b) fail.
"""

import re
from pathlib import Path

import numpy as np
import pytest

SRC = Path(__file__).resolve().parents[1] / "paper_1304_1755_amd" / "csrc" / "sg_mg.hip"


def _constants():
    s = SRC.read_text()
    def get(name):
        return int(re.search(name + r" = (\d+)", s).group(1))
    return get("kTileCX"), get("kTileCY"), get("kTileHX"), get("kTileHY"), get("kTileR")


TCX, TCY, HX, HY, R = _constants()
P = R + 2

# CPU emulation of the single-mode tile kernels (down: nu forward sweeps + residual + restriction;
# up: prolongation + nu backward sweeps) against the same steps on the whole grid
def colours(reverse):
    qs = [0, 1, 2, 3]
    return qs[::-1] if reverse else qs
def cpar(q): return ((q & 1) ^ 1, (q >> 1) ^ 1)  # (x parity, y parity)
def relax_global(u, f, st, rd, nx, q):
    px, py = cpar(q)
    up = np.zeros((nx + 2, nx + 2)); up[1:-1, 1:-1] = u
    new = u.copy()
    for y in range(py, nx, 2):
        for x in range(px, nx, 2):
            c = up[y:y + 3, x:x + 3]
            s = st[y, x]
            acc = f[y, x]
            acc -= s[0] * c[0, 0] + s[1] * c[0, 1] + s[2] * c[0, 2]
            acc -= s[6] * c[2, 0] + s[7] * c[2, 1] + s[8] * c[2, 2]
            acc -= s[3] * c[1, 0] + s[5] * c[1, 2]
            new[y, x] = acc * rd[y, x]
    return new
def restrict_value(get, X, Y):
    fx, fy = 2 * X + 1, 2 * Y + 1
    acc = 0.0
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            w = 0.25 if (dx and dy) else (1.0 if dx == 0 else 0.5) * (1.0 if dy == 0 else 0.5)
            acc += w * get(fx + dx, fy + dy)
    return acc
def prolong_value(get, nxc, x, y):
    if x & 1: cx = [(x - 1) >> 1]; wx = 1.0
    else: cx = [(x >> 1) - 1, x >> 1]; wx = 0.5
    if y & 1: cy = [(y - 1) >> 1]; wy = 1.0
    else: cy = [(y >> 1) - 1, y >> 1]; wy = 0.5
    acc = 0.0
    for Y in cy:
        if Y < 0 or Y >= nxc: continue
        for X in cx:
            if X < 0 or X >= nxc: continue
            acc += get(X, Y)
    return wx * wy * acc
def residual(u, f, st, nx):
    up = np.zeros((nx + 2, nx + 2)); up[1:-1, 1:-1] = u
    r = np.zeros_like(u)
    for y in range(nx):
        for x in range(nx):
            c = up[y:y + 3, x:x + 3]; s = st[y, x]; acc = f[y, x]
            for dy in range(3):
                for dx in range(3):
                    acc -= s[dy * 3 + dx] * c[dy, dx]
            r[y, x] = acc
    return r
def tile_down(f, st, rd, nx, nu):
    nxc = (nx - 1) // 2
    ntx, nty = -(-nxc // TCX), -(-nxc // TCY)
    uo = np.full((nx, nx), np.nan); fc = np.full((nxc, nxc), np.nan)
    for by in range(nty):
        for bx in range(ntx):
            X0, Y0 = bx * TCX, by * TCY
            rx0, ry0 = 2 * X0 - HX, 2 * Y0 - HY
            u = np.zeros((P, P))
            def inn(gx, gy): return 0 <= gx < nx and 0 <= gy < nx
            for sw in range(nu):
                for q in colours(False):
                    px, py = cpar(q)
                    new = u.copy()
                    for t in range(R * R // 4):
                        lx = 2 * (t % (R // 2)) + px; ly = 2 * (t // (R // 2)) + py
                        gx, gy = rx0 + lx, ry0 + ly
                        assert 0 <= lx < R and 0 <= ly < R
                        if not inn(gx, gy): continue
                        c = u[ly:ly + 3, lx:lx + 3]; s = st[gy, gx]
                        acc = f[gy, gx]
                        acc -= s[0] * c[0, 0] + s[1] * c[0, 1] + s[2] * c[0, 2]
                        acc -= s[6] * c[2, 0] + s[7] * c[2, 1] + s[8] * c[2, 2]
                        acc -= s[3] * c[1, 0] + s[5] * c[1, 2]
                        new[ly + 1, lx + 1] = acc * rd[gy, gx]
                    u = new
            r = np.zeros((2 * TCY + 1, 2 * TCX + 1))
            for t in range(R * R // 4):
                for q in range(4):
                    px, py = cpar(q)
                    lx = 2 * (t % (R // 2)) + px; ly = 2 * (t // (R // 2)) + py
                    gx, gy = rx0 + lx, ry0 + ly
                    ax, ay = gx - 2 * X0, gy - 2 * Y0
                    if inn(gx, gy) and 0 <= ax <= 2 * TCX and 0 <= ay <= 2 * TCY:
                        c = u[ly:ly + 3, lx:lx + 3]; s = st[gy, gx]; acc = f[gy, gx]
                        for dy in range(3):
                            for dx in range(3): acc -= s[dy * 3 + dx] * c[dy, dx]
                        r[ay, ax] = acc
            for i in range(TCX * TCY):
                X, Y = X0 + i % TCX, Y0 + i // TCX
                if X < nxc and Y < nxc:
                    fc[Y, X] = restrict_value(lambda x, y: r[y - 2 * Y0, x - 2 * X0], X, Y)
            cx1 = nx if X0 + TCX >= nxc else 2 * (X0 + TCX)
            cy1 = nx if Y0 + TCY >= nxc else 2 * (Y0 + TCY)
            for t in range(R * R // 4):
                for q in range(4):
                    px, py = cpar(q)
                    lx = 2 * (t % (R // 2)) + px; ly = 2 * (t // (R // 2)) + py
                    gx, gy = rx0 + lx, ry0 + ly
                    if 2 * X0 <= gx < cx1 and 2 * Y0 <= gy < cy1:
                        assert np.isnan(uo[gy, gx])
                        uo[gy, gx] = u[ly + 1, lx + 1]
    return uo, fc
def tile_up(f, st, rd, ui, ec, nx, nu):
    nxc = (nx - 1) // 2
    ntx, nty = -(-nxc // TCX), -(-nxc // TCY)
    uo = np.full((nx, nx), np.nan)
    for by in range(nty):
        for bx in range(ntx):
            X0, Y0 = bx * TCX, by * TCY
            rx0, ry0 = 2 * X0 - HX, 2 * Y0 - HY
            u = np.zeros((P, P))
            def inn(gx, gy): return 0 <= gx < nx and 0 <= gy < nx
            for t in range(R * R // 4):
                for q in range(4):
                    px, py = cpar(q)
                    lx = 2 * (t % (R // 2)) + px; ly = 2 * (t // (R // 2)) + py
                    gx, gy = rx0 + lx, ry0 + ly
                    if inn(gx, gy):
                        u[ly + 1, lx + 1] = ui[gy, gx] + prolong_value(lambda X, Y: ec[Y, X], nxc, gx, gy)
            for sw in range(nu):
                for q in colours(True):
                    px, py = cpar(q)
                    new = u.copy()
                    for t in range(R * R // 4):
                        lx = 2 * (t % (R // 2)) + px; ly = 2 * (t // (R // 2)) + py
                        gx, gy = rx0 + lx, ry0 + ly
                        if not inn(gx, gy): continue
                        c = u[ly:ly + 3, lx:lx + 3]; s = st[gy, gx]
                        acc = f[gy, gx]
                        acc -= s[0] * c[0, 0] + s[1] * c[0, 1] + s[2] * c[0, 2]
                        acc -= s[6] * c[2, 0] + s[7] * c[2, 1] + s[8] * c[2, 2]
                        acc -= s[3] * c[1, 0] + s[5] * c[1, 2]
                        new[ly + 1, lx + 1] = acc * rd[gy, gx]
                    u = new
            cx1 = nx if X0 + TCX >= nxc else 2 * (X0 + TCX)
            cy1 = nx if Y0 + TCY >= nxc else 2 * (Y0 + TCY)
            for t in range(R * R // 4):
                for q in range(4):
                    px, py = cpar(q)
                    lx = 2 * (t % (R // 2)) + px; ly = 2 * (t // (R // 2)) + py
                    gx, gy = rx0 + lx, ry0 + ly
                    if 2 * X0 <= gx < cx1 and 2 * Y0 <= gy < cy1:
                        assert np.isnan(uo[gy, gx])
                        uo[gy, gx] = u[ly + 1, lx + 1]
    return uo


def _problem(nx, seed):
    rng = np.random.default_rng(seed)
    st = rng.uniform(-0.3, -0.05, (nx, nx, 9))
    st[:, :, 4] = rng.uniform(2.5, 3.0, (nx, nx))
    return st, 1.0 / st[:, :, 4], rng.standard_normal((nx, nx)), rng.standard_normal(((nx - 1) // 2, (nx - 1) // 2))


def test_geometry_covers_the_region():
    assert 2 * TCX + 2 * HX == R and 2 * TCY + 2 * HY == R


@pytest.mark.parametrize("nx", [63, 127])
def test_tiles_equal_whole_grid_steps(nx):
    st, rd, f, ec = _problem(nx, nx)
    nu = 2
    u = np.zeros((nx, nx))
    for sw in range(nu):
        for q in colours(False):
            u = relax_global(u, f, st, rd, nx, q)
    r = residual(u, f, st, nx)
    nxc = (nx - 1) // 2
    fcr = np.array([[restrict_value(lambda x, y: r[y, x], X, Y) for X in range(nxc)] for Y in range(nxc)])
    uo, fc = tile_down(f, st, rd, nx, nu)
    assert not np.isnan(uo).any() and not np.isnan(fc).any()
    assert np.array_equal(uo, u) and np.array_equal(fc, fcr)
    v = u.copy()
    for y in range(nx):
        for x in range(nx):
            v[y, x] += prolong_value(lambda X, Y: ec[Y, X], nxc, x, y)
    for sw in range(nu):
        for q in colours(True):
            v = relax_global(v, f, st, rd, nx, q)
    uo2 = tile_up(f, st, rd, u, ec, nx, nu)
    assert not np.isnan(uo2).any()
    assert np.array_equal(uo2, v)
