"""The parity harness itself, on the CPU: the active-set comparison of the GPU tests
accepts equal lists and, on a mismatch, names each differing slot with its activation
value against delta0 (the report a real mismatch would give)."""
import numpy as np
import pytest

import oracle
import scenes
from test_gpu_parity import assert_same_active, plane_activation


def test_active_set_report_names_the_slot_and_its_activation():
    b = scenes.robot_batch(2, seed=1)
    P = scenes.solver_params(k_max=64)
    q, u, lam = b.q0.copy(), b.u0.copy(), np.zeros(b.n_lam)
    ref = oracle.step_forward(b, P, q, u, lam, np.zeros(b.n_ctrl))
    assert_same_active(b, P, q, u, {k: v.copy() for k, v in ref.items()}, ref, "equal")
    # the host-side activation value decides every ground-plane slot as the oracle did
    for w in range(b.n_worlds):
        s0 = b.slot_off[w]
        act = set(ref["act_slot"][s0:s0 + ref["n_act"][w]].tolist())
        for s in range(b.slot_off[w + 1] - s0):
            a = plane_activation(b, P, q, u, w, s)
            if a is not None:
                assert (a <= P["delta0"]) == (s in act), (w, s, a)
    w = 1
    s0, n = b.slot_off[w], ref["n_act"][w]
    assert n >= 2
    got = {k: v.copy() for k, v in ref.items()}
    dropped = int(got["act_slot"][s0 + n - 1])
    got["act_slot"][s0 + n - 1] = -1
    got["n_act"][w] = n - 1
    with pytest.raises(AssertionError) as e:
        assert_same_active(b, P, q, u, got, ref, "planted")
    msg = str(e.value)
    assert f"world {w} slot {dropped}: oracle only" in msg
    a = plane_activation(b, P, q, u, w, dropped)
    if a is not None:
        # an active slot passed the activation test at q-
        assert a <= P["delta0"]
        assert "%.6e" % a in msg
