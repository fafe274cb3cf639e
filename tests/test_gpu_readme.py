"""The Python example of the README runs as printed and gives a finite, moving flow."""
import os
import re

import numpy as np
import pytest

from helpers import log_case

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_python_example_runs():
    with open(os.path.join(ROOT, "README.md")) as f:
        blocks = re.findall(r"```python\n(.*?)```", f.read(), re.S)
    assert len(blocks) == 1
    log_case("README example")
    ns = {}
    exec(compile(blocks[0], "README.md", "exec"), ns)
    for k in ("rho", "ux", "uy", "uz", "F", "T", "x", "U", "W"):
        assert np.all(np.isfinite(ns[k])), k
    assert ns["x"].shape == (1, 2)
    assert ns["uz"].shape == (64, 64, 128)  # the 3-D solve's fields, [nz][ny][nx]
    assert ns["ux"].mean() > 0.0  # driven by the body force
