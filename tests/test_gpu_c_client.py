"""The C-ABI from plain C: tests/c_client/step_client (built by build())
reads a mesh, creates a plan, computes the reference and takes one step in a
uniform velocity field, with HIP runtime calls for memory only; at the reference
shape the step is dt u0 for every node.  Run as a child process."""
import os
import subprocess

import numpy as np
import pytest

from paper_1612_03399_amd import workload as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
CLIENT = os.path.join(HERE, "c_client", "step_client")


def test_c_client_step(tmp_path):
    assert os.path.exists(CLIENT), "the C client is not built (run __graft_entry__.build())"
    v, faces = W.icosphere(2)
    X = 0.5 + 0.2 * v
    e4 = W.edges4_from_faces(faces)
    mesh = tmp_path / "drop.txt"
    with open(mesh, "w") as fh:
        fh.write(f"{len(X)} {len(e4)} {len(faces)}\n")
        np.savetxt(fh, X, fmt="%.17g")
        np.savetxt(fh, faces, fmt="%d")
        np.savetxt(fh, e4, fmt="%d")
    r = subprocess.run([CLIENT, str(mesh)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert "nodes 162" in r.stdout
