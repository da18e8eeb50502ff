"""The literal workload constants of paper_2304_04214_amd.synthetic, re-derived
with the oracle's wall law: u_tau u+(Re_tau) = U_c at the centreline (y+ = Re_tau,
Reichardt law, Sec. II.C Eq. (16)), nu0 = u_tau delta / Re_tau, tau0 = 1/2 + 3 nu0
(Eq. (5)) with delta = ny / 2."""
import pytest

import oracle as O
from paper_2304_04214_amd import synthetic as S


@pytest.mark.parametrize("name", sorted(S.WORKLOADS))
def test_workload_constants(name):
    w = S.WORKLOADS[name]
    if w["re_tau"] is None:  # the oracle configuration gives tau0 directly
        assert w["tau0"] == 0.52
        return
    u_tau = S.U_C / O.uplus(w["re_tau"])
    assert abs(w["u_tau"] / u_tau - 1) < 1e-14
    tau0 = 0.5 + 3 * u_tau * (w["ny"] / 2) / w["re_tau"]
    assert abs(w["tau0"] - tau0) < 1e-15


@pytest.mark.parametrize("re_tau", sorted(S.U_TAU_OF_RE))
def test_friction_velocity_table(re_tau):
    assert abs(S.U_TAU_OF_RE[re_tau] * O.uplus(re_tau) / S.U_C - 1) < 1e-14
