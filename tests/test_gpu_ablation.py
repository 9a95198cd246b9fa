"""The ablation module on a short soft-cube curve (GPU).

j_max = 0 is NCG without preconditioning (Sec. 3.2), so it takes no inner
iterations. On this soft magnet the preconditioned form needs fewer
nonlinear iterations than the plain one (Table 1's trend), every beta* and the
(t1)-(t3) rule reach their stopping test, and the torque tolerance holds at the
end of every field.
"""
import pytest

pytestmark = pytest.mark.gpu


def test_ablation_rows_on_soft_cube(capsys):
    from paper_1801_03690_amd import ablation
    rows = ablation.main(["--workload", "soft_cube", "--fields", "3", "--jmax", "0,4", "--beta", "1,2",
                          "--tau-f", "1e-10", "--max-nli", "5000"])
    by = {r["setting"]: r for r in rows}
    plain, prec = by["jmax=0, beta*ZA"], by["jmax=4, beta*ZA"]
    assert plain["li"] == 0 and prec["li"] > 0
    assert prec["nli"] < plain["nli"], (prec["nli"], plain["nli"])
    for r in rows:
        assert r["rc"] == 0 and r["max_status"] == 0, r
    for r in (plain, prec, by["jmax=4, beta*FR"], by["jmax=4, beta*PRP"]):
        assert r["torque_max"] < 1e-6, r
    out = capsys.readouterr().out
    assert out.count("\n| jmax=") == len(rows)
