"""Pins of the oracle's unit-diagonal form of Algorithm 3 and of its
fixed-point tables (Section III: the loop needs no division, so its tables
suit a fixed-point word; the bit depth is left open).  Each test ties the
new functions to something other than themselves: the pinned fase() on the
same block, the Cauchy-Schwarz bound, hand-worked rounding cases, the error
bound of round-to-nearest, and a table whose entries are dyadic so that its
16-bit words are exact."""
import numpy as np
import pytest

import oracle
from paper_2204_14194_amd import synth


def _block(M=16, N=16, seed=5):
    img = synth.synth_image(48, 48, seed=seed)
    b = synth.Block(0, 8, 10, 5, 6, 6, 5)
    lost = synth.lost_mask(48, 48, [b])
    s, sup = oracle.area_signal(img, lost, b.y0, b.x0, M, N)
    return s, oracle.area_weights(M, N, 0.8, sup), b


def test_unit_form_equals_algorithm3():
    """fase_unit on D C D gives fase()'s selections (up to parallel atoms)
    and model."""
    phi = synth.dictionary(16, 16, ("dct", "wht"))
    s, w, _ = _block()
    C, D = oracle.table_generation(phi, w)
    cls = oracle.duplicate_classes(phi)
    ref = oracle.fase(s, w, phi, C, D, 0.5, 60, cls)
    got = oracle.fase_unit(s, w, phi, oracle.unit_table(C, D), D, 0.5, 60, cls)
    # parallel atoms (the two constant atoms) tie: rounding picks either
    np.testing.assert_array_equal(cls[got.sel], cls[ref.sel])
    np.testing.assert_allclose(got.coef, ref.coef, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(got.g, ref.g, atol=1e-9)
    np.testing.assert_allclose(got.best, ref.best, rtol=1e-9)
    np.testing.assert_allclose(got.energy, ref.energy, rtol=1e-9)
    # a forced run follows the forced atoms
    forced = ref.sel[::-1].copy()
    f1 = oracle.fase(s, w, phi, C, D, 0.5, 60, cls, forced=forced)
    f2 = oracle.fase_unit(s, w, phi, oracle.unit_table(C, D), D, 0.5, 60, cls, forced=forced)
    np.testing.assert_allclose(f2.g, f1.g, atol=1e-9)
    np.testing.assert_allclose(f2.picked, f1.picked, rtol=1e-9)


def test_unit_table_is_bounded_by_one():
    """|D_k C_kl D_l| <= 1 (Cauchy-Schwarz in the weighted product), with a
    unit diagonal wherever the atom has a nonzero weighted norm."""
    phi = synth.dictionary(16, 16, ("dct", "gauss"), n_gauss=256)
    _, w, _ = _block()
    C, D = oracle.table_generation(phi, w)
    G = oracle.unit_table(C, D)
    assert np.abs(G).max() <= 1.0 + 1e-12
    np.testing.assert_allclose(np.diag(G)[D > 0], 1.0, atol=1e-12)


def test_quantise_rounding_cases():
    step = 2.0 ** -14
    G = np.array([1.0, -1.0, 0.0, step, -step, 2.5 * step, 3.5 * step, -2.5 * step,
                  0.5 * step, 1.5 * step, 1.999 * step, 2.0 - step, -2.0])
    q = oracle.quantise_table(G)
    assert q.dtype == np.int16
    np.testing.assert_array_equal(q, [16384, -16384, 0, 1, -1, 2, 4, -2, 0, 2, 2, 32767, -32768])
    with pytest.raises(ValueError):
        oracle.quantise_table(np.array([2.0]))
    with pytest.raises(ValueError):
        oracle.quantise_table(np.array([1j]))
    # other word lengths follow the same rule
    np.testing.assert_array_equal(oracle.quantise_table(np.array([0.3, -0.7]), 4), [5, -11])


def test_quantise_error_bound():
    """Round to nearest: every word is within half a step of its entry, and
    the nearest word (no neighbour is closer)."""
    rng = np.random.default_rng(8)
    G = rng.uniform(-1.0, 1.0, size=20000)
    q = oracle.quantise_table(G).astype(np.float64)
    step = 2.0 ** -14
    err = np.abs(q * step - G)
    assert err.max() <= step / 2
    assert (np.abs((q + 1) * step - G) >= err).all() and (np.abs((q - 1) * step - G) >= err).all()


def test_dyadic_table_words_are_exact():
    """Walsh-Hadamard atoms (entries +-1/16 on a 16 x 16 area) under 0/1
    weights with 128 support pixels: every C_kl is a multiple of 1/256 and
    C_kk = 1/2, so D C D holds multiples of 1/128 and its 14-bit words are
    exact (D C D = 2 C up to the rounding of D = 1/sqrt(1/2)); the run on
    the words is then the run on the exact table 2 C."""
    phi = synth.dictionary(16, 16, ("wht",))
    w = np.zeros(256)
    w[np.random.default_rng(2).permutation(256)[:128]] = 1.0
    C, D = oracle.table_generation(phi, w)
    np.testing.assert_array_equal(np.diag(C), 0.5)
    exact = 2.0 * C
    np.testing.assert_array_equal(np.rint(exact * 256), exact * 256)
    G = oracle.unit_table(C, D)
    assert np.abs(G - exact).max() < 1e-15
    q = oracle.quantise_table(G)
    np.testing.assert_array_equal(q.astype(np.float64) * 2.0 ** -14, exact)
    s = synth.synth_image(16, 16, seed=4).reshape(-1).astype(np.float64) * w
    a = oracle.fase_unit(s, w, phi, exact, D, 0.5, 40)
    b = oracle.fase_unit(s, w, phi, q.astype(np.float64) * 2.0 ** -14, D, 0.5, 40)
    np.testing.assert_array_equal(a.sel, b.sel)
    np.testing.assert_array_equal(a.g, b.g)


def test_fixed_point_run_stays_close():
    """On the benchmark geometry's dictionary (16 x 16 here) the run on the
    words differs from the exact run by far less than a grey level where it
    follows the same atoms, and the first selections agree (the table error
    is at most 2**-15 per entry)."""
    phi = synth.dictionary(16, 16, ("dct", "wht"))
    s, w, b = _block()
    C, D = oracle.table_generation(phi, w)
    G = oracle.unit_table(C, D)
    Gq = oracle.quantise_table(G).astype(np.float64) * 2.0 ** -14
    assert np.abs(Gq - G).max() <= 2.0 ** -15
    ex = oracle.fase_unit(s, w, phi, G, D, 0.5, 60)
    fx = oracle.fase_unit(s, w, phi, Gq, D, 0.5, 60)
    cls = oracle.duplicate_classes(phi)
    eq = cls[ex.sel] == cls[fx.sel]
    assert eq[:10].all()
    same = int(np.argmin(eq)) if not eq.all() else 60
    run = oracle.fase_unit(s, w, phi, Gq, D, 0.5, same)
    ref = oracle.fase_unit(s, w, phi, G, D, 0.5, same)
    assert np.abs(run.g - ref.g).max() < 0.05
