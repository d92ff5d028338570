"""Pins of the oracle's quantizers (Section 3.2, Eq. 2-3, zone-2 rule, byte
layout) by hand-worked boundary tables and invariants."""
import numpy as np
import pytest

from conftest import read_golden

AMP = dict(step_f=0.25, step_c=2.0, T=16.0)


def _table(name):
    fwd, inv = [], []
    for row in read_golden(name):
        parts = row.split()
        if parts[0] == "D":
            inv.append(tuple(float(v) for v in parts[1:]))
        else:
            fwd.append((float(parts[0]), int(parts[1])))
    return fwd, inv


def test_amplitude_boundary_table(O):
    fwd, inv = _table("amp_quant_boundaries.txt")
    for c, s in fwd:
        assert O.quant_amp(c, **AMP) == s, (c, s)
    for s, v, z in inv:
        assert O.dequant_amp(int(s), **AMP) == v
        assert O.zone_amp(int(s), **AMP) == int(z)


@pytest.mark.parametrize("params", [AMP, dict(step_f=1.0, step_c=8.0, T=16.0)])
def test_amplitude_invariants(O, params):
    cs = np.linspace(-2000, 2000, 40001)
    syms = np.array([O.quant_amp(c, **params) for c in cs])
    assert np.all(np.diff(syms) >= 0), "monotone non-decreasing"
    vals = np.array([O.dequant_amp(s, **params) for s in range(256)])
    assert np.all(np.diff(vals) > 0), "levels strictly increasing"
    # odd symmetry of the reconstruction magnitudes (where both sides exist)
    for m in range(128):
        assert vals[128 + m] == -vals[128 - m]
    # idempotence: quantizing a reconstruction point returns its level
    for s in range(256):
        assert O.quant_amp(vals[s], **params) == s
    # error <= half a step inside the representable range
    lo, hi = vals[0], vals[255]
    for c in cs[(cs >= lo) & (cs <= hi)][::7]:
        s = O.quant_amp(c, **params)
        step = params["step_f"] if abs(c) <= params["T"] else params["step_c"]
        assert abs(vals[s] - c) <= step / 2 + 1e-12
    # zone 0 is exactly the zero level, zones 1/2 split at T
    for s in range(256):
        z = O.zone_amp(s, **params)
        if s == 128:
            assert z == 0 and vals[s] == 0
        else:
            assert z == (1 if abs(vals[s]) <= params["T"] else 2)


def test_deadzone_boundary_table(O):
    p = O.QuantParams("paper", 32, 16, B1=0, B2=16, mu=50.0, alpha1=0.1, A0=1.0, A1=10.0)
    fwd, inv = _table("deadzone_boundaries.txt")
    for c, s in fwd:
        assert O.quant_paper(c, 3, p) == s, (c, s)
    for s, v in inv:
        assert abs(O.dequant_paper(int(s), 3, p) - v) < 1e-12


def test_mulaw_boundary_table(O):
    p = O.QuantParams("paper", 32, 16, B1=16, B2=16, mu=50.0, alpha1=0.004, A0=2.0, A1=1.0)
    fwd, inv = _table("mulaw_boundaries.txt")
    for c, s in fwd:
        assert O.quant_paper(c, 0, p) == s, (c, s)
    for s, v in inv:
        assert abs(O.dequant_paper(int(s), 0, p) - v) < 1e-12


@pytest.mark.parametrize("zone_bin", [0, 1])
def test_paper_quantizer_invariants(O, zone_bin):
    # bins [0, B1) mu-law, [B1, B2) deadzone
    p = O.QuantParams("paper", 32, 16, B1=1, B2=8, mu=50.0, alpha1=0.004, A0=3.0, A1=2.0)
    k = 0 if zone_bin == 0 else 4
    A = p.A0 if zone_bin == 0 else p.A1
    cs = np.linspace(-1.5 * A, 1.5 * A, 6001)
    syms = np.array([O.quant_paper(c, k, p) for c in cs])
    assert np.all(np.diff(syms) >= 0)
    assert syms[0] == 0 and syms[-1] == 255
    vals = np.array([O.dequant_paper(s, k, p) for s in range(256)])
    assert np.all(np.diff(vals[129:]) > 0) and np.all(np.diff(vals[:128]) > 0)
    assert vals[128] == 0.0 and vals[127] <= 0 and vals[129] >= 0
    # idempotence on every level away from the zero level.  Levels 127 and 129
    # reconstruct on the edge of the zero level (+-d1 for Eq. 3, 0 for Eq. 2),
    # which the strict inequalities of Eq. 3 (and c = 0 for Eq. 2) send to 128.
    for s in list(range(0, 127)) + list(range(130, 256)):
        assert O.quant_paper(vals[s], k, p) == s, s
    edge = 0.0 if zone_bin == 0 else p.alpha1 * p.A1
    assert vals[129] == edge and vals[127] == -edge
    assert O.quant_paper(vals[129], k, p) == 128 and O.quant_paper(vals[127], k, p) == 128
    # the reconstruction is within half a level spacing of c inside [-A, A]
    for c in cs[np.abs(cs) <= A][::11]:
        s = O.quant_paper(c, k, p)
        if zone_bin == 1 and abs(c) <= p.alpha1 * p.A1:
            assert s == 128
            continue
        nb = [vals[t] for t in (s - 1, s, s + 1) if 0 <= t < 256]
        spacing = max(abs(nb[i + 1] - nb[i]) for i in range(len(nb) - 1))
        assert abs(vals[s] - c) <= spacing / 2 + 1e-9 or (zone_bin == 0 and abs(c) < vals[130])


def test_zone2_is_always_zero(O):
    p = O.QuantParams("paper", 32, 16, B1=2, B2=8, mu=50.0, alpha1=0.004, A0=3.0, A1=2.0)
    for k in range(8, 16):
        for c in (-1e6, -1.0, 0.0, 1e-9, 7.0, 1e6):
            assert O.quant_paper(c, k, p) == 128
        assert all(O.dequant_paper(s, k, p) == 0.0 for s in range(256))
        assert all(O.zone(s, k, p) == 2 for s in range(256))
    assert O.zone(17, 0, p) == 0 and O.zone(17, 1, p) == 0 and O.zone(17, 2, p) == 1 and O.zone(17, 7, p) == 1


# Stream-level encode side (Section 3.1 transform, Section 3.2 quantizer,
# Section 3.3 histogram): each is the composition of pinned pieces, checked
# here against that composition written out, plus numpy's own routines.

@pytest.mark.parametrize("kind,N,E", [("amp", 16, 16), ("amp", 64, 20), ("paper", 32, 16)])
def test_quantize_stream_is_the_per_coefficient_quantizer_of_the_window_transform(O, kind, N, E):
    rng = np.random.default_rng(70 + N + E)
    x = (rng.standard_normal(3 * N + 5) * 4.0).astype(np.float32)
    if kind == "amp":
        p = O.QuantParams("amp", N, E, **AMP)
    else:
        p = O.QuantParams("paper", N, E, B1=2, B2=E, mu=50.0, alpha1=0.004, A0=9.0, A1=5.0)
    coef = O.dct_stream(x, N, E).reshape(-1, E)
    want = np.empty(coef.shape, dtype=np.uint8)
    for w in range(coef.shape[0]):
        for k in range(E):
            c = float(coef[w, k])
            want[w, k] = O.quant_amp(c, p.step_f, p.step_c, p.T) if kind == "amp" else O.quant_paper(c, k, p)
    assert np.array_equal(O.quantize_stream(x, p), want.ravel())


def test_histogram_equals_bincount(O):
    rng = np.random.default_rng(71)
    for n in (0, 1, 257, 10000):
        sym = rng.integers(0, 256, size=n, dtype=np.uint8)
        sym[: n // 3] = 128  # a dominant symbol, as the quantizers give
        assert np.array_equal(O.histogram(sym), np.bincount(sym, minlength=256).astype(np.uint64))


def test_zone_maxima_are_order_statistics_of_the_zones(O):
    # the linear percentile at 0 / 100 is the zone's min / max of |c|, and
    # between two order statistics it interpolates (checked on a tiny case
    # by sorting by hand)
    N, E, B1, B2 = 16, 8, 2, 6
    rng = np.random.default_rng(72)
    x = (rng.standard_normal(5 * N) * 3.0).astype(np.float32)
    p = O.QuantParams("paper", N, E, B1=B1, B2=B2, mu=50.0, alpha1=0.004, A0=1.0, A1=1.0)
    coef = np.abs(O.dct_stream(x, N, E).reshape(-1, E))
    z0, z1 = np.sort(coef[:, :B1].ravel()), np.sort(coef[:, B1:B2].ravel())
    assert O.paper_zone_maxima(x, p, 100.0) == (z0[-1], z1[-1])
    assert O.paper_zone_maxima(x, p, 0.0) == (z0[0], z1[0])
    q = 99.9
    for z, got in zip((z0, z1), O.paper_zone_maxima(x, p, q)):
        pos = q / 100.0 * (z.size - 1)
        i = int(np.floor(pos))
        want = z[i] + (pos - i) * (z[min(i + 1, z.size - 1)] - z[i])
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want))
