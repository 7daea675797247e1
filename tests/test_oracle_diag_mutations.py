"""The post-processing pins must catch plausible mistakes in ``oracle/diag.py``.

Each case plants one mistake in a copy of the module's source, loads the copy
as a separate module, and runs every check of ``test_oracle_diag`` on it: at
least one must fail. The real module is untouched.
"""
import os
import types

import pytest

from tests import test_oracle_diag as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "diag.py")

MUTANTS = [
    ("coefficient without the 1/2", "q = 0.5 * rho * u * u * length", "q = rho * u * u * length"),
    ("crossing interpolated from the wrong end", "frac = -s[k] / (s[k + 1] - s[k])",
     "frac = s[k + 1] / (s[k + 1] - s[k])"),
    ("crossing counted one too many", "period = (t[-1] - t[0]) / (len(t) - 1)", "period = (t[-1] - t[0]) / len(t)"),
    ("mean not removed", "    s = s - s.mean()\n", "    s = s\n"),
    ("downward crossings", "if s[k] < 0.0 <= s[k + 1]:", "if s[k] >= 0.0 > s[k + 1]:"),
    ("drag amplitude not halved", '"cd_amp": float((cd.max() - cd.min()) / 2.0)', '"cd_amp": float(cd.max() - cd.min())'),
    ("lift amplitude from the drag", '"cl_amp": float((cl.max() - cl.min()) / 2.0)',
     '"cl_amp": float((cd.max() - cd.min()) / 2.0)'),
    ("wake length over the radius", "return (x_end - rear) / (2.0 * radius)", "return (x_end - rear) / radius"),
    ("wake measured from the centre", "rear = cx + radius", "rear = cx"),
    ("wake axis from the lower row only", "return float((1.0 - w) * ux[j, i] + w * ux[j + 1, i])",
     "return float(ux[j, i])"),
    ("wake end from the wrong side", "x_end = i + prev / (prev - nxt)", "x_end = i + nxt / (prev - nxt)"),
    ("separation on the body radius", "r = radius + offset", "r = radius"),
    ("tangent side ignored", "return -np.sin(th) * vx + side * np.cos(th) * vy",
     "return -np.sin(th) * vx + np.cos(th) * vy"),
    ("separation from the upper half only", "return float(0.5 * (found[0] + found[1]))", "return float(found[0])"),
    ("bilinear with x weight in y", "return float(bot + fy * (top - bot))", "return float(bot + fx * (top - bot))"),
    ("lower half not mirrored", "y = cy + side * r * np.sin(th)", "y = cy + r * np.sin(th)"),
]


def _load(source: str) -> types.ModuleType:
    mod = types.ModuleType("diag_mutant")
    exec(compile(source, "diag_mutant.py", "exec"), mod.__dict__)
    return mod


def _caught(mod) -> bool:
    for check in pins.CHECKS:
        try:
            check(mod)
        except Exception:
            return True
    return False


def test_real_module_passes_every_check():
    assert not _caught(_load(open(SRC).read()))


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not found once: {name}"
    assert _caught(_load(src.replace(old, new))), f"mutant not caught: {name}"
