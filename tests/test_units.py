"""The physical-units front end (sscn_units_to_g, host only) against the
oracle's independent derivation (numerical quadrature of the frozen
directions' ground states) and against fixed numbers: the oscillator
length of 87Rb in a 100 Hz trap."""
import math

import pytest

import oracle
from paper_1605_03958_amd import sscn

RB87 = 86.909180527            # atomic mass of 87Rb, u
A_RB87 = 100.4                 # its s-wave scattering length, Bohr radii (a commonly used value)


def test_oscillator_length_of_rb87_at_100_hz():
    """l = sqrt(hbar/(m omega)) = 1.0784 um for 87Rb at omega = 2 pi x 100 Hz."""
    _, l, t = sscn.units_to_g(3, 1000, A_RB87, RB87, 2 * math.pi * 100.0)
    assert abs(l - 1.07843e-6) < 2e-10
    assert abs(t - 1 / (2 * math.pi * 100.0)) < 1e-15
    _, lo, _ = oracle.units_to_g(3, 1000, A_RB87, RB87, 2 * math.pi * 100.0)
    assert abs(l / lo - 1) < 1e-14


@pytest.mark.parametrize("dim,tight", [(3, (1.0, 1.0)), (2, (20.0, 1.0)), (2, (3.7, 1.0)), (1, (50.0, 80.0)),
                                       (1, (10.0, 10.0))])
@pytest.mark.parametrize("atoms,a", [(1000, A_RB87), (2.5e5, 5.3), (300, -10.0)])
def test_nonlinearity_matches_the_oracle(dim, tight, atoms, a):
    g, _, _ = sscn.units_to_g(dim, atoms, a, RB87, 2 * math.pi * 60.0, tight)
    go, _, _ = oracle.units_to_g(dim, atoms, a, RB87, 2 * math.pi * 60.0, tight)
    assert abs(g - go) <= 1e-12 * abs(go)
    assert (g > 0) == (a > 0)


def test_nonlinearity_scales_with_atoms_and_length():
    g1, _, _ = sscn.units_to_g(2, 1000, 50.0, RB87, 2 * math.pi * 50.0, (8.0, 1.0))
    g2, _, _ = sscn.units_to_g(2, 3000, 50.0, RB87, 2 * math.pi * 50.0, (8.0, 1.0))
    g3, _, _ = sscn.units_to_g(2, 1000, 25.0, RB87, 2 * math.pi * 50.0, (8.0, 1.0))
    assert abs(g2 / g1 - 3) < 1e-14 and abs(g3 / g1 - 0.5) < 1e-14


@pytest.mark.parametrize("bad", [dict(dim=0), dict(dim=4), dict(atoms=0.0), dict(mass=-1.0), dict(omega=0.0),
                                 dict(dim=2, tight=(0.0, 1.0)), dict(dim=1, tight=(1.0, float("nan")))])
def test_invalid_inputs_are_refused(bad):
    args = dict(dim=3, atoms=1000.0, a=50.0, mass=RB87, omega=100.0, tight=(1.0, 1.0))
    args.update(bad)
    with pytest.raises(sscn.SSCNError) as e:
        sscn.units_to_g(args["dim"], args["atoms"], args["a"], args["mass"], args["omega"], args["tight"])
    assert e.value.code == sscn.E_INVALID
