"""Host logic of the learned-surrogate pipeline: unpacking a flat parameter vector
(the packing gnmpc.gnn_flat gives gnmpc_gnn_loss_grad and gnmpc_adam_step) back
into GNN weights."""
import numpy as np
import pytest

from paper_2602_17601_amd import workloads as wl

sur = pytest.importorskip("paper_2602_17601_amd.surrogate")
gn = pytest.importorskip("paper_2602_17601_amd.gnmpc")


@pytest.mark.parametrize("Hd,L", [(16, 1), (32, 3)])
def test_unflat_inverts_flat(Hd, L):
    W = wl.gnn_weights(3, Hd, L, dt=0.02, bias_scale=0.5)
    theta = gn.gnn_flat(W)
    V = sur.gnn_unflat(theta, W)
    assert V.Hd == Hd and V.L == L and V.dt == W.dt
    np.testing.assert_array_equal(gn.gnn_flat(V), theta)
    # each block lands in its own place: a change of one entry shows up only there
    theta2 = theta.copy()
    k = W.W_enc.size + W.b_enc.size + 5      # entry 5 of round 0's edge matrix
    theta2[k] += 1.0
    V2 = sur.gnn_unflat(theta2, W)
    assert V2.W_edge[0].reshape(-1)[5] == W.W_edge[0].reshape(-1)[5] + 1.0
    np.testing.assert_array_equal(V2.W_enc, W.W_enc)
    np.testing.assert_array_equal(V2.W_dec, W.W_dec)


def test_unflat_rejects_a_wrong_size():
    W = wl.gnn_weights(3, 16, 2)
    with pytest.raises(ValueError):
        sur.gnn_unflat(np.zeros(gn.gnn_flat(W).size + 1), W)
