"""Host-side parts of the learned preconditioner (no GPU): the library's
FP64 training targets against the oracle's, and the weight packing."""
import numpy as np
import pytest

from oracle import precond as opc


def _params(pse, n, L, xi=0.5, rc=6.0):
    return pse.Params(n, L, 1.0, 1.0, 1.0, xi, rc, 32, 8, 0.0, 1e-4, 32, 2, 1, 0)


def test_library_targets_match_oracle():
    import paper_1611_09322_amd as pse
    import synth

    x, L = synth.hard_spheres(150, 0.2, seed=21)
    idx = np.array([0, 17, 42, 99, 149], dtype=np.int32)
    got = pse.pse_precond_targets(_params(pse, len(x), L), x, idx)
    ref = opc.targets(x, idx, L, 1.0, 1.0, 0.5, 6.0)
    np.testing.assert_allclose(got, ref, atol=1e-10, rtol=1e-10)


def test_library_targets_isolated_and_custom_radius():
    import paper_1611_09322_amd as pse

    L = 20.0
    x = np.array([[2.0, 2.0, 2.0], [12.0, 12.0, 12.0], [12.0, 14.5, 12.0]])
    got = pse.pse_precond_targets(_params(pse, 3, L), x, np.array([0, 1], np.int32))
    np.testing.assert_allclose(got[0], np.eye(3), atol=1e-12)
    ref = opc.targets(x, [1], L, 1.0, 1.0, 0.5, 6.0, radius=3.0)
    got = pse.pse_precond_targets(_params(pse, 3, L), x, np.array([1], np.int32), radius=3.0)
    np.testing.assert_allclose(got, ref, atol=1e-12)


def test_targets_reject_bad_index():
    import paper_1611_09322_amd as pse

    with pytest.raises(pse.PSEError):
        pse.pse_precond_targets(_params(pse, 3, 20.0), np.zeros((3, 3)), np.array([3], np.int32))


def test_weight_pack_roundtrip_and_bf16_bits():
    from paper_1611_09322_amd import precond as ppc

    w = opc.init_weights(3, scale=0.4)
    flat = ppc.pack(w)
    assert flat.size == 7312
    back = ppc.unpack(flat)
    for k in w:
        np.testing.assert_allclose(back[k], w[k].astype(np.float32), rtol=0, atol=0)
    bits = ppc.bf16_bits(flat)
    vals = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    np.testing.assert_array_equal(vals, opc.bf16_round(flat))
    # padding entries are zero
    assert not np.any(flat.reshape(-1)[0:64 * 32].reshape(64, 32)[:, 24:])
