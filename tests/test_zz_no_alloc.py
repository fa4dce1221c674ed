"""GPU: the entry point without allocation, m1_dynamic_c_tilde_noalloc,
against m1_dynamic_c_tilde (whose workspace argument it replaces by the
library's static device array) through the C ABI: two calls in a row, the
second on a smaller grid, each bitwise equal to the workspace entry point's
value on the same inputs (a maximum over cells: exact), and both equal to the
oracle's to rounding."""
import numpy as np
import pytest

from oracle import m1_oracle as M
from paper_2606_02711_amd import inputs

pytestmark = pytest.mark.gpu


def _sound_speed(T, mu=1.22, gamma=5.0 / 3.0):
    return np.sqrt(gamma * M.K_B * np.asarray(T) / (mu * M.M_H))


def test_noalloc_dynamic_c_tilde_equals_workspace_entry_point():
    from paper_2606_02711_amd import m1
    big = inputs.config2()                                     # 524288 cells: 1024 blocks
    small = inputs.random_small("cyl", 41, 57, 6, log_nHI=(-4.0, 3.0))
    for name, p, c_prev in (("config2 512x1024", big, 0.0), ("random 41x57", small, 3.0e7)):
        cs = _sound_speed(p["fields"]["T"])
        print(f"[gpu] dynamic c_tilde noalloc vs workspace: {name}", flush=True)
        got = m1.dynamic_c_tilde(p, cs, c_prev, noalloc=True)
        want = m1.dynamic_c_tilde(p, cs, c_prev)
        assert got == want, (name, got, want)
        assert got == pytest.approx(M.dynamic_c_tilde(p, cs, c_prev), rel=1e-13)


def test_noalloc_reports_a_bad_temperature():
    from paper_2606_02711_amd import m1
    p = inputs.random_small("cart", 12, 9, 7)
    p["fields"]["T"][4, 5] = 0.0
    print("[gpu] dynamic c_tilde noalloc with T = 0 in a cell", flush=True)
    with pytest.raises(m1.M1Error):
        m1.dynamic_c_tilde(p, np.full((9, 12), 1.0e5), noalloc=True)
