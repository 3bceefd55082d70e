"""The two v half-steps between steps composed in Fourier space, checked on the CPU.

Between two Strang steps the closing v half-step of one and the opening one of
the next apply the same circulant A (Section 1.2: the cyclic shift by b after
the kernel w_q(s)) and add the same delta-f source s (Section 3.1), so
u2 = A (A u0 + s) + s.  The composed launch evaluates that on two real lines
packed as one complex line z = uA + i uB:

  U = P Z + Q conj(Z_{N-m}) + Zs,  W = Q Z + P conj(Z_{N-m}) + conj(Zs_{N-m}),
  y = IFFT(P U + Q W),  P = (S_A + S_B) / 2,  Q = (S_A - S_B) / 2,

with S the kernel's symbol, zs each line's source taken at the positions j - b
its first store would have used, the result stored at twice the shift and the
source added there.  This test checks that identity with numpy against the two
half-steps applied in turn as plain circular sums; it exercises no library code.
"""
import numpy as np
import pytest


def _half_step(u, w, d, b, src):
    # (A u)_i = sum_q w_q u_{i+b+q}, q = -d .. d+1, then the source
    out = np.zeros_like(u)
    for qi, wq in enumerate(w):
        out += wq * np.roll(u, -(b + qi - d))
    return out + src


def _symbol(w, d, n):
    m = np.arange(n)
    q = np.arange(len(w)) - d
    return (w[None, :] * np.exp(2j * np.pi * np.outer(m, q) / n)).sum(axis=1)


def _composed(uA, uB, wA, wB, d, bA, bB, sA, sB):
    n = len(uA)
    SA, SB = _symbol(wA, d, n), _symbol(wB, d, n)
    P, Q = (SA + SB) / 2, (SA - SB) / 2
    j = np.arange(n)
    Z = np.fft.fft(uA + 1j * uB)
    Zs = np.fft.fft(sA[(j - bA) % n] + 1j * sB[(j - bB) % n])
    partner = (-j) % n
    Zp, Sp = np.conj(Z[partner]), np.conj(Zs[partner])
    U = P * Z + Q * Zp + Zs
    W = Q * Z + P * Zp + Sp
    y = np.fft.ifft(P * U + Q * W)
    # unshifted index j goes to position j - 2b, the source added there
    return y.real[(j + 2 * bA) % n] + sA, y.imag[(j + 2 * bB) % n] + sB


def _lagrange(d, s):
    nodes = np.arange(-d, d + 2)
    w = np.ones(len(nodes))
    for i, q in enumerate(nodes):
        for k in nodes:
            if k != q:
                w[i] *= (s - k) / (q - k)
    return w


@pytest.mark.parametrize("n,d", [(16, 1), (64, 4), (256, 8)])
@pytest.mark.parametrize("bA,bB", [(0, 0), (3, -5), (-40, 17)])
def test_composed_equals_two_half_steps(n, d, bA, bB):
    rng = np.random.default_rng([n, d, bA + 100, bB + 100])
    uA, uB = rng.standard_normal(n), rng.standard_normal(n)
    sA, sB = 0.1 * rng.standard_normal(n), 0.1 * rng.standard_normal(n)
    wA, wB = _lagrange(d, 0.3), _lagrange(d, 0.85)
    refA = _half_step(_half_step(uA, wA, d, bA, sA), wA, d, bA, sA)
    refB = _half_step(_half_step(uB, wB, d, bB, sB), wB, d, bB, sB)
    gotA, gotB = _composed(uA, uB, wA, wB, d, bA, bB, sA, sB)
    assert np.max(np.abs(gotA - refA)) < 1e-12 * max(1.0, np.max(np.abs(refA)))
    assert np.max(np.abs(gotB - refB)) < 1e-12 * max(1.0, np.max(np.abs(refB)))


def test_composed_without_source_is_the_kernel_squared():
    # no source: y = IFFT(P2 Z + Q2 conj(Z_{N-m})), P2 = P^2 + Q^2, Q2 = 2 P Q
    n, d = 128, 8
    rng = np.random.default_rng(3)
    uA, uB = rng.standard_normal(n), rng.standard_normal(n)
    wA, wB = _lagrange(d, 0.1), _lagrange(d, 0.6)
    SA, SB = _symbol(wA, d, n), _symbol(wB, d, n)
    P, Q = (SA + SB) / 2, (SA - SB) / 2
    Z = np.fft.fft(uA + 1j * uB)
    Zp = np.conj(Z[(-np.arange(n)) % n])
    y = np.fft.ifft((P * P + Q * Q) * Z + 2 * P * Q * Zp)
    zero = np.zeros(n)
    assert np.allclose(y.real, _half_step(_half_step(uA, wA, d, 0, zero), wA, d, 0, zero), atol=1e-12)
    assert np.allclose(y.imag, _half_step(_half_step(uB, wB, d, 0, zero), wB, d, 0, zero), atol=1e-12)
