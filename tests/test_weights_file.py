"""The shipped network file is self-consistent (CPU only)."""
import json
import os

import numpy as np

import pdegen as g

import pytest

WDIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2305_16432_amd",
                    "weights")


@pytest.mark.parametrize("fname,ordering,h,n_mp,dm", [
    ("heat3d_h32_mp3.npz", 0, 32, 3, 1), ("heat3d_h32_mp3_color.npz", 1, 32, 3, 1),
    ("heat3d_h32_mp3_frobenius.npz", 0, 32, 3, 1), ("heat3d_h32_mp3_ft64.npz", 0, 32, 3, 1),
    ("heat3d_h32_mp3_color3.npz", 1, 32, 3, 3), ("heat3d_h32_mp1_color3.npz", 1, 32, 1, 3),
    ("fem2d_h64_mp5.npz", 0, 64, 5, 1)])
def test_weights_file_layout(fname, ordering, h, n_mp, dm):
    W = np.load(os.path.join(WDIR, fname))  # allow_pickle stays False
    assert (int(W["h"]), int(W["n_mp"]), int(W["diag_mode"]), int(W["ordering"])) == (h, n_mp, dm, ordering)
    n = sum(int(np.prod(s)) for _, s in g.gnn_param_shapes(h, n_mp))
    assert W["params"].shape == (n,) and np.all(np.isfinite(W["params"]))
    log = json.loads(str(W["log"]))
    assert int(W["best_iters"]) < log["jacobi_iters"]


def test_fine_tuned_network_provenance():
    """The 64^3 fine-tuning started from the shipped 32^3 network."""
    W = np.load(os.path.join(WDIR, "heat3d_h32_mp3_ft64.npz"))
    cfg = json.loads(str(W["config"]))
    assert cfg["m"] == 64 and cfg["init"].endswith("heat3d_h32_mp3.npz") and cfg["loss"] == "data"


def test_oracle_triples_provenance():
    """The networks trained since the triple generator came in name a triples
    file (written by the oracle's PCG) as their training data."""
    for fname in ("heat3d_h32_mp3_color3.npz", "heat3d_h32_mp1_color3.npz", "fem2d_h64_mp5.npz"):
        cfg = json.loads(str(np.load(os.path.join(WDIR, fname))["config"]))
        assert cfg["triples"].endswith(".npz") and "m" not in cfg
