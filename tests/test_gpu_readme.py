"""The README's Python example runs as written (bank, trigger reduction,
planner, serving loop)."""
import os
import re

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_python_example_runs(capsys):
    text = open(os.path.join(ROOT, "README.md"), encoding="utf-8").read()
    blocks = re.findall(r"```python\n(.*?)```", text, flags=re.S)
    assert len(blocks) == 1
    exec(compile(blocks[0], "README.md", "exec"), {"__name__": "readme_example"})
    out = capsys.readouterr().out.split()
    assert len(out) >= 2 and float(out[-1]) > 0.0  # the serving run's p99 latency in ms
