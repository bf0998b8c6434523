"""The FP64 tanh of the device code (tanh_d, and tanh_d_tab with its table of
2^(j/32)) emulated on the CPU with every FP64 operation rounded once (fma
exactly, through rationals) and the hardware reciprocal estimate perturbed
by its worst relative error either way (4.6e-8 measured on gfx950): the
absolute error against a 50-digit tanh stays below 5e-16, and the table
entries are the correctly rounded powers.  The constants are read from the
device sources, so the check follows any change to them."""
import math
import random
import re
from decimal import Decimal, getcontext
from fractions import Fraction as Fr
from pathlib import Path

import pytest

CSRC = Path(__file__).resolve().parents[1] / "paper_2410_22867_amd" / "csrc"
RCP_ERR = 4.6e-8
NUM = r"(-?[0-9][0-9.e+-]*)"


def _fma(a, b, c):
    return float(Fr(a) * Fr(b) + Fr(c))


def _mul(a, b):
    return float(Fr(a) * Fr(b))


def _body(src, name):
    i = src.index(name + "(double x")
    return src[i:src.index("\n}", i)]


def _consts(body):
    scale = float(re.search(r"fabs\(x\) \* " + NUM, body).group(1))
    kmul = float(re.search(r"rint\(u \* " + NUM, body).group(1))
    head, tail = [float(v) for v in re.findall(r"fma\(-(?:n|k), " + NUM + r", (?:-u|w)\)", body)]
    p0 = float(re.search(r"double p = " + NUM + ";", body).group(1))
    coefs = [float(v) for v in re.findall(r"p = fma\(p, w, " + NUM + r"\);", body)]
    return scale, kmul, head, tail, [p0] + coefs


def _finish(x, e, eps):
    d = float(Fr(1) + Fr(e))
    q0 = float(Fr(1) / Fr(d)) * (1.0 + eps)
    r = _fma(-d, q0, 1.0)
    q = _fma(q0, _fma(r, r, r), q0)
    return math.copysign(_fma(2.0, q, -1.0), x)


def _poly(cs, w):
    p = cs[0]
    for c in cs[1:]:
        p = _fma(p, w, c)
    return p


def tanh_d(x, c, eps):
    scale, kmul, head, tail, cs = c
    u = min(max(_mul(abs(x), scale), 0.0), 1.0)
    n = float(round(_mul(u, kmul)))
    w = _fma(-n, tail, _fma(-n, head, -u))
    return _finish(x, math.ldexp(_poly(cs, w), int(n)), eps)


def tanh_d_tab(x, c, tab, eps):
    scale, kmul, head, tail, cs = c
    u = min(max(_mul(abs(x), scale), 0.0), 1.0)
    k = float(round(_mul(u, kmul)))
    w = _fma(-k, tail, _fma(-k, head, -u))
    ki = int(k)
    return _finish(x, math.ldexp(_mul(_poly(cs, w), tab[ki & 31]), ki >> 5), eps)


@pytest.fixture(scope="module")
def forms():
    dev = (CSRC / "dp_device.h").read_text()
    emb = (CSRC / "k_embed.hip").read_text()
    tab_src = re.search(r"kExp2Frac32\[32\] = \{([^}]*)\}", emb).group(1)
    tab = [float(v) for v in re.findall(r"[0-9][0-9.e+-]*", tab_src)]
    return _consts(_body(dev, "tanh_d")), _consts(_body(dev, "tanh_d_tab")), tab


def test_table_is_correctly_rounded(forms):
    getcontext().prec = 50
    _, _, tab = forms
    assert len(tab) == 32
    for j, t in enumerate(tab):
        ref = Decimal(2) ** (Decimal(j) / 32)
        assert abs(Decimal(t) - ref) <= ref * Decimal(2) ** -53


@pytest.mark.parametrize("form", ["tanh_d", "tanh_d_tab"])
def test_fp64_tanh_error_bound(forms, form):
    getcontext().prec = 50
    c_plain, c_tab, tab = forms
    rng = random.Random(11)
    xs = [rng.uniform(-40, 40) for _ in range(600)] + [rng.uniform(-3, 3) for _ in range(600)] + \
         [10 ** rng.uniform(-8, 0) * rng.choice((-1, 1)) for _ in range(400)] + [0.0, 32.0, -32.0, 1e3]
    worst = 0.0
    for x in xs:
        e2 = (Decimal(x) * 2).exp()
        ref = (e2 - 1) / (e2 + 1)
        for eps in (RCP_ERR, -RCP_ERR, 0.0):
            y = tanh_d(x, c_plain, eps) if form == "tanh_d" else tanh_d_tab(x, c_tab, tab, eps)
            worst = max(worst, abs(float(Decimal(y) - ref)))
    assert worst < 5e-16, worst
