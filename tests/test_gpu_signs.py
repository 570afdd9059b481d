"""DSRG_OPT_CHECK_SIGNS: every CCVV work item's contribution to E_CCVV is <= 0
when all denominators e_i + e_j - e_a - e_b are negative (Eq. expensive:
R(Delta) <= 0 and x^2 - x y + y^2 >= 0). With ordered orbital energies the
check word stays 0 in every entry point and precision, and the energies are
bitwise those of a call without the option; with the virtual energies moved
below the core ones (every denominator positive, which the library does not
forbid) every entry point sets bit 0, and a call without the option does not."""
import numpy as np
import pytest
import torch

from paper_1603_00561_amd.workloads import make_problem

pytestmark = pytest.mark.gpu


def _b():
    from paper_1603_00561_amd import binding
    return binding


def _dev(p, flip=False):
    eps_v = p.eps_v - (p.eps_v.max() - p.eps_c.min() + 1.0) if flip else p.eps_v
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()  # noqa: E731
    return [t(p.B_cv), t(p.B_ca), t(p.B_av), t(p.eps_c), t(p.eps_a), t(eps_v), t(p.gamma1),
            p.s]


def _calls(args, precision):
    b = _b()
    gE = torch.tensor([1.0, 0.5, -0.25], dtype=torch.float64, device="cuda")
    return {
        "energy": lambda chk: b.energy(*args, precision=precision, check_signs=chk),
        "noalloc": lambda chk: b.energy_noalloc(*args, precision=precision, check_signs=chk),
        "backward": lambda chk: b.energy_backward(*args, gE, precision=precision,
                                                  check_signs=chk)["E"],
    }


@pytest.mark.parametrize("precision", ["fp64", "ozaki"])
@pytest.mark.parametrize("shape", [(3, 2, 70, 40), (5, 1, 150, 33)])
def test_ordered_energies_pass_and_results_unchanged(precision, shape):
    b = _b()
    p = make_problem(*shape, s=0.5, seed=sum(shape) + 61)
    args = _dev(p)
    b.sign_check()   # clear
    for name, call in _calls(args, precision).items():
        print(f"[gpu-signs] {precision} {shape} {name}", flush=True)
        E0 = call(False)
        E1 = call(True)
        assert torch.equal(E0, E1), name
        assert b.sign_check() == 0, name


@pytest.mark.parametrize("precision", ["fp64", "ozaki"])
def test_positive_denominators_set_the_word(precision):
    b = _b()
    p = make_problem(3, 2, 70, 40, s=0.5, seed=62)
    args = _dev(p, flip=True)
    b.sign_check()
    for name, call in _calls(args, precision).items():
        print(f"[gpu-signs] flipped {precision} {name}", flush=True)
        E = call(False)
        assert float(E[0]) > 0.0            # every CCVV term is now positive
        assert b.sign_check() == 0, name    # not checked without the option
        call(True)
        assert b.sign_check() == 1, name
        assert b.sign_check() == 0, name    # cleared by the read
