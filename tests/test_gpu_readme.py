"""The README's Python example runs as written (steps, then a gradient through the rollout)."""

import os
import re

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.timeout(300)
def test_readme_example_runs():
    with open(os.path.join(ROOT, "README.md"), encoding="utf-8") as f:
        blocks = re.findall(r"```python\n(.*?)```", f.read(), flags=re.S)
    assert len(blocks) == 1
    env = {}
    exec(compile(blocks[0], "README.md", "exec"), env)
    h, e0, infos = env["h"], env["e0"], env["infos"]
    assert all(i["iters"] > 0 and i["rel_res"] <= 1e-9 for i in infos)
    for g in (h.grad, e0.grad):
        assert g is not None and bool(torch.isfinite(g).all()) and float(g.abs().max()) > 0.0
