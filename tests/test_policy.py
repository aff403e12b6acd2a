"""The learned -> IC(0) -> Jacobi fallback policy (paper_2305_16432_amd/
policy.py) on the CPU, behind a scripted backend that exists only here."""
import pytest

from paper_2305_16432_amd import policy


class ScriptedBackend:
    """Plays back outcomes: check -> (ok, bad_row); ic0 -> None (pivot
    breakdown after every shift) or a factor; pcg[stage] -> status."""

    def __init__(self, check=(True, -1), ic0_ok=True, pcg=None):
        self._check, self._ic0_ok = check, ic0_ok
        self._pcg = pcg or {}
        self.calls = []

    def predict(self, S, net, b):
        self.calls.append("predict")
        return "Lnet", "Unet"

    def check(self, S, l_val):
        self.calls.append("check")
        assert l_val == "Lnet"
        return self._check

    def ic0(self, S, max_retries):
        self.calls.append("ic0")
        return ("Lic", "Uic", 2e-3) if self._ic0_ok else None

    def pcg(self, S, kind, b, l_val, ut_val, tol, maxit, max_restarts):
        stage = {"Lnet": "learned", "Lic": "ic0", None: "jacobi"}[l_val]
        assert kind == ("jacobi" if stage == "jacobi" else "llt")
        self.calls.append("pcg:" + stage)
        st = self._pcg.get(stage, policy.OK)
        return f"x_{stage}", {"status": st, "iters": {"learned": 20, "ic0": 35, "jacobi": 100}[stage],
                              "relres_true": 1e-7 if st == policy.OK else 1e-2}


NET = {"params": None, "h": 32, "n_mp": 3, "diag_mode": 1}


def test_learned_factor_used_when_valid_and_converging():
    be = ScriptedBackend()
    x, rep = policy.solve("S", "b", NET, backend=be)
    assert x == "x_learned" and rep.stage == "learned" and rep.iters == 20
    assert be.calls == ["predict", "check", "pcg:learned"]
    assert rep.tried == [("learned", "converged")]


def test_rejected_factor_falls_back_to_ic0_without_solving():
    be = ScriptedBackend(check=(False, 17))
    x, rep = policy.solve("S", "b", NET, backend=be)
    assert x == "x_ic0" and rep.stage == "ic0" and rep.shift == 2e-3
    assert be.calls == ["predict", "check", "ic0", "pcg:ic0"]
    assert rep.tried[0] == ("learned", "factor rejected at row 17")


@pytest.mark.parametrize("status,why", [(policy.EBREAKDOWN, "breakdown"), (policy.ENOTCONV, "not converged")])
def test_learned_solve_failure_falls_back(status, why):
    be = ScriptedBackend(pcg={"learned": status})
    x, rep = policy.solve("S", "b", NET, backend=be)
    assert rep.stage == "ic0" and x == "x_ic0"
    assert rep.tried == [("learned", why), ("ic0", "converged")]


def test_ic0_breakdown_then_jacobi():
    be = ScriptedBackend(ic0_ok=False)
    x, rep = policy.solve("S", "b", None, backend=be)
    assert x == "x_jacobi" and rep.stage == "jacobi"
    assert be.calls == ["ic0", "pcg:jacobi"]
    assert rep.tried == [("ic0", "pivot breakdown after every shift"), ("jacobi", "converged")]


def test_every_stage_failing_reports_no_stage():
    be = ScriptedBackend(pcg={"learned": policy.ENOTCONV, "ic0": policy.EBREAKDOWN,
                              "jacobi": policy.ENOTCONV})
    x, rep = policy.solve("S", "b", NET, backend=be)
    assert rep.stage == "" and rep.status == policy.ENOTCONV and x == "x_jacobi"
    assert [t[0] for t in rep.tried] == ["learned", "ic0", "jacobi"]


def test_without_network_starts_at_ic0():
    be = ScriptedBackend()
    _, rep = policy.solve("S", "b", None, backend=be)
    assert rep.stage == "ic0" and "predict" not in be.calls
