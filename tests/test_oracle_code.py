"""Pins of the oracle's code construction, CRC, encoder and channel.

Each check compares the oracle with something it does not share code with:
the paper's Fig. 1 netlist, explicit Kronecker powers, catalogue CRC values,
Python big-integer polynomial division, Gaussian log-densities, and Monte
Carlo estimates of the quantities the Gaussian approximation approximates.
"""
import binascii
import os

import numpy as np
import pytest

import oracle as O
from paper_1609_09358_amd import inputs
from tests import _bruteforce as BF

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_fig1():
    stages, frozen, N = [], [], None
    with open(os.path.join(GOLDEN, "fig1_encoder_n8.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if not line:
                continue
            if line[0] == "N":
                N = int(line[1])
            elif line[0] == "frozen":
                frozen = [int(v) for v in line[1:]]
            elif line[0] == "stage":
                stages.append(tuple(int(v) for v in line[1:]))
    return N, frozen, stages


# ---------------------------------------------------------------- encoder

def test_encoder_matches_fig1_netlist():
    """Simulate the Fig. 1 circuit gate by gate for all 256 inputs."""
    N, _, stages = _read_fig1()
    for word in range(2 ** N):
        u = np.array([(word >> (N - 1 - i)) & 1 for i in range(N)], np.uint8)
        v = u.copy()
        for s in sorted({st[0] for st in stages}):
            for (_, a, b) in [st for st in stages if st[0] == s]:
                v[a] ^= v[b]
        assert np.array_equal(O.polar_transform(u), v), word


def test_fig1_corner_outputs():
    """x_7 = u_7 and x_0 = XOR of all u (Fig. 1)."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        u = rng.integers(0, 2, 8).astype(np.uint8)
        x = O.polar_transform(u)
        assert x[7] == u[7]
        assert x[0] == np.bitwise_xor.reduce(u)


@pytest.mark.parametrize("N", [2, 4, 16, 128, 1024])
def test_encoder_equals_kronecker_power(N):
    rng = np.random.default_rng(N)
    for _ in range(8):
        u = rng.integers(0, 2, N).astype(np.uint8)
        assert np.array_equal(O.polar_transform(u), BF.encode_matrix(u))


@pytest.mark.parametrize("N", [8, 256, 2048])
def test_encoder_is_an_involution(N):
    """G G = I over GF(2), so encoding twice returns u."""
    rng = np.random.default_rng(7 + N)
    u = rng.integers(0, 2, N).astype(np.uint8)
    assert np.array_equal(O.polar_transform(O.polar_transform(u)), u)


def test_build_u_places_info_then_crc_ascending():
    fr = O.ga_frozen(64, 24, 2.0, 16 / 64)
    info = inputs.info_bits(1, 16, seed=3)[0]
    u = O.build_u(info, 16, 8, 0x07, fr)
    free = np.where(fr == 0)[0]
    assert np.all(u[fr == 1] == 0)
    assert np.array_equal(u[free[:16]], info)
    assert np.array_equal(u[free[16:]], O.crc(info, 8, 0x07))


# ---------------------------------------------------------------- construction

def test_fig1_frozen_set_from_ga():
    """Fig. 1 freezes u_0, u_1, u_2, u_4 (info set {3, 5, 6, 7}) for N = 8, k = 4."""
    N, frozen, _ = _read_fig1()
    for ebn0 in (0.0, 2.0, 4.0):
        fr = O.ga_frozen(N, 4, ebn0, 0.5)
        assert sorted(np.where(fr == 1)[0].tolist()) == frozen


@pytest.mark.parametrize("N,ebn0", [(128, 2.0), (1024, 2.5), (2048, 2.0)])
def test_ga_partial_order(N, ebn0):
    """A channel whose index is a bitwise superset of another's is at least as
    reliable (the plus transform never loses to the minus transform).  Below
    x = 0.0294 the two-piece approximation of phi exceeds 1 and the minus
    transform collapses to 0, so the order is checked where m > 0.03; the
    collapsed channels are always far fewer than the frozen ones."""
    m = O.ga_means(N, O.sigma2(ebn0, 0.5))
    idx = np.arange(N)
    for i in range(0, N, max(1, N // 64)):
        if m[i] <= 0.03:
            continue
        sup = idx[(idx & i) == i]
        assert np.all(m[sup] >= m[i] * (1 - 1e-12))
    assert (m == 0).sum() < N // 8


def test_ga_single_step_against_monte_carlo():
    """One polarisation step: the GA means of the check and variable sides
    against the empirical means of boxplus(a, b) and a + b for a, b drawn from
    the consistent Gaussian N(m, 2m) (the approximation's own premise)."""
    rng = np.random.default_rng(11)
    for m0 in (0.8, 3.0, 8.0):
        s2 = 2.0 / m0  # channel mean 2 / sigma^2 = m0
        m = O.ga_means(2, s2)
        a = rng.normal(m0, np.sqrt(2 * m0), 400000)
        b = rng.normal(m0, np.sqrt(2 * m0), 400000)
        box = 2 * np.arctanh(np.clip(np.tanh(a / 2) * np.tanh(b / 2), -1 + 1e-15, 1 - 1e-15))
        assert abs(m[1] - 2 * m0) < 1e-12
        assert abs(m[0] - box.mean()) / box.mean() < 0.06, (m0, m[0], box.mean())


def test_ga_phi_against_its_definition():
    """phi(x) = 1 - E[tanh(u/2)], u ~ N(x, 2x): the GA check step reduces to
    phi^{-1}(1 - (1 - phi(m))^2); check that the N = 2 minus mean satisfies that
    relation with phi evaluated by numerical integration (within the accuracy
    of the two-piece approximation)."""
    t = np.linspace(-60, 60, 200001)

    def phi(x):
        if x <= 0:
            return 1.0
        pdf = np.exp(-(t - x) ** 2 / (4 * x)) / np.sqrt(4 * np.pi * x)
        return 1.0 - np.trapezoid(np.tanh(t / 2) * pdf, t)

    for m0 in (1.0, 4.0, 12.0):
        mm = O.ga_means(2, 2.0 / m0)[0]
        lhs = phi(mm)
        rhs = 1 - (1 - phi(m0)) ** 2
        assert abs(lhs - rhs) / rhs < 0.08, (m0, lhs, rhs)


# ---------------------------------------------------------------- CRC

def _catalogue():
    rows = []
    with open(os.path.join(GOLDEN, "crc_check_values.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if line and line[0] != "name":
                rows.append((line[0], int(line[1]), int(line[2], 16), int(line[3], 16)))
    return rows


def _bits_of(data: bytes) -> np.ndarray:
    return np.unpackbits(np.frombuffer(data, np.uint8))


def _val(bits) -> int:
    v = 0
    for b in bits:
        v = (v << 1) | int(b)
    return v


@pytest.mark.parametrize("row", _catalogue(), ids=lambda r: r[0])
def test_crc_catalogue_check_values(row):
    name, width, poly, check = row
    assert _val(O.crc(_bits_of(b"123456789"), width, poly)) == check


def test_crc16_matches_binascii():
    rng = np.random.default_rng(5)
    for n in (1, 7, 64, 131):
        data = rng.integers(0, 256, n, dtype=np.uint8).tobytes()
        assert _val(O.crc(_bits_of(data), 16, 0x1021)) == binascii.crc_hqx(data, 0)


@pytest.mark.parametrize("width,poly", [(8, 0x07), (16, 0x1021), (24, 0x864CFB)])
def test_crc_is_polynomial_remainder(width, poly):
    """M(x) x^c mod P(x) by Python big-integer division over GF(2)."""
    rng = np.random.default_rng(width)
    P = (1 << width) | poly
    for nbits in (1, 5, 64, 512, 1536):
        bits = rng.integers(0, 2, nbits).astype(np.uint8)
        m = _val(bits) << width
        while m.bit_length() > width:
            m ^= P << (m.bit_length() - width - 1)
        assert _val(O.crc(bits, width, poly)) == m


def test_crc_linearity():
    rng = np.random.default_rng(9)
    a = rng.integers(0, 2, 512).astype(np.uint8)
    b = rng.integers(0, 2, 512).astype(np.uint8)
    assert np.array_equal(O.crc(a ^ b, 24, 0x864CFB), O.crc(a, 24, 0x864CFB) ^ O.crc(b, 24, 0x864CFB))


# ---------------------------------------------------------------- channel

def test_channel_llr_is_log_likelihood_ratio():
    """LLR = ln p(y|x=0) / p(y|x=1) for BPSK (0 -> +1, 1 -> -1) in Gaussian noise."""
    sig2 = O.sigma2(2.5, 0.5)
    x = inputs.info_bits(1, 4096, seed=2)[0]
    z = inputs.noise(1, 4096, seed=2)[0]
    llr = O.channel_llr(x, z, sig2)
    y = (1.0 - 2.0 * x) + np.sqrt(sig2) * z
    lp0 = -((y - 1.0) ** 2) / (2 * sig2)
    lp1 = -((y + 1.0) ** 2) / (2 * sig2)
    np.testing.assert_allclose(llr, (lp0 - lp1).astype(np.float32), rtol=1e-6, atol=1e-6)


def test_sigma2_matches_snr_definition():
    """Es = 1 per BPSK symbol, Eb = Es / R, N0 = 2 sigma^2."""
    for ebn0, R in ((2.0, 0.5), (2.5, 0.5), (1.0, 0.25), (3.0, 0.75)):
        s2 = O.sigma2(ebn0, R)
        eb_n0 = (1.0 / R) / (2.0 * s2)
        assert abs(10 * np.log10(eb_n0) - ebn0) < 1e-12
