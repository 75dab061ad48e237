"""Checks of the seeded synthetic-input generator."""
import numpy as np

from paper_0911_1407_amd import synth


def test_deterministic_and_integral_counts():
    a = synth.config_instance("plain32")
    b = synth.config_instance("plain32")
    assert np.array_equal(a["counts"], b["counts"]) and np.array_equal(a["s_true"], b["s_true"])
    assert np.all(a["counts"] == np.round(a["counts"])) and np.all(a["counts"] >= 0)


def test_amplitude_gives_requested_variance():
    n, box, sigma = (32, 32, 32), (100.0,) * 3, 1.0
    pk = synth.power_shape_half(n, box)
    amp = synth.amplitude_for_sigma(pk, n, box, sigma)
    # ensemble variance of a cell = (1/V) sum over all grid modes of A pk
    c = synth.hermitian_multiplicity(n)
    assert abs(np.sum(c * amp * pk) / 1e6 - sigma ** 2) < 1e-12
    # sample variance of a realisation is close to the ensemble value
    inst = synth.config_instance("plain32")
    g = inst["s_true"] + 0.5 * sigma ** 2
    assert abs(g.mean()) < 1e-12
    assert 0.7 < g.var() < 1.3


def test_block_mask_fraction():
    inst = synth.make_instance((32, 32, 32), (64.0,) * 3, 1.0, 1.0, radius=1e9, mask_frac=0.2, seed=0)
    zero_blocks = (inst["w"].reshape(4, 8, 4, 8, 4, 8) == 0).all(axis=(1, 3, 5)).sum()
    assert zero_blocks == round(0.2 * 64)
    assert np.all(inst["counts"][inst["w"] == 0] == 0)


def test_batch_instances():
    insts = synth.batch_instances(count=8)
    assert len(insts) == 8
    for it in insts:
        assert it["n"][0] in (32, 48, 64, 96)
        assert 0.1 <= it["nbar"] <= 5.0 and 0.8 <= it["sigma"] <= 1.8
