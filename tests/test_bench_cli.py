"""Host-side checks of bench.py and the input generator (no GPU)."""
import os
import subprocess
import sys

import numpy as np

from paper_1905_01381_amd import flops, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_batch_molecule_generator_is_per_index():
    """Molecule i of the 64-molecule set depends on (seed, i) only."""
    sizes = inputs.c4_sizes()
    assert sizes.shape == (64,) and sizes.min() >= 10 and sizes.max() <= 120
    for i in (0, 5, 63):
        a = inputs.c4_molecule(i)
        b = inputs.c4_molecule(i)
        assert len(a.mol.shell_l) == 6 * sizes[i]
        assert np.array_equal(a.mol.atoms, b.mol.atoms)
        assert np.array_equal(a.orbitals, b.orbitals)


def test_flop_model_grows_with_angular_momentum():
    f = [flops.per_quartet(*c, nJ=1, nK=1) for c in [(0, 0, 0, 0), (1, 0, 0, 0), (1, 1, 1, 1), (2, 2, 2, 2)]]
    assert all(x > 0 for x in f) and f == sorted(f)
