"""The threshold autotuner: it times the caller's workload under candidate
settings, keeps only faster settings whose solutions agree with the
reference, and leaves them installed; the tuned factorization solves as the
default one does."""

import numpy as np
import pytest

from workloads import convdiff2d_upwind

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1712_07297_amd as P

    P.lib()
    P.config_reset()
    yield P
    P.config_reset()


def test_autotune_keeps_a_valid_setting(P):
    from paper_1712_07297_amd.autotune import CANDIDATES, autotune

    systems = []
    for side, pe in ((96, 20.0), (128, 60.0)):
        A = convdiff2d_upwind(side, pe, 0.5)
        systems.append((A.row_ptr, A.col_idx, A.val, (side, side, 1)))
    n = sum(len(s[0]) - 1 for s in systems)
    B = torch.tensor(np.random.default_rng(0).uniform(-1, 1, (1, n)), device="cuda")
    lines = []
    chosen = autotune(systems, 1e-3, 64, symmetric=0, B=B, krylov="gmres", repeats=1, log=lines.append)
    print("\n".join(lines), flush=True)
    assert set(chosen) == set(CANDIDATES)
    for name, v in chosen.items():
        assert v in CANDIDATES[name] or v == P.config_get(name)
        assert P.config_get(name) == v
    # the tuned setting solves as the default one does
    F = P.Factor.batch(systems, 1e-3, 64, symmetric=0)
    x, it, rel, ok = F.gmres(B, 1e-10, 300, 30)
    P.config_reset()
    F0 = P.Factor.batch(systems, 1e-3, 64, symmetric=0)
    x0, it0, rel0, ok0 = F0.gmres(B, 1e-10, 300, 30)
    assert ok and ok0 and abs(it - it0) <= 1
    assert torch.linalg.norm(x - x0) / torch.linalg.norm(x0) < 1e-8
