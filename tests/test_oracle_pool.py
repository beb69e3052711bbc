"""The pooled direction sums (tests/oracle_pool.py) equal the serial oracle (no GPU)."""
import numpy as np

from oracle.formal import formal_solution
from oracle.levels import Level
from oracle.rates import zero_radiation
from paper_1701_01607_amd import synth
from tests.oracle_pool import pooled_formal_solution, pooled_norm


def test_pooled_formal_solution_equals_the_serial_one():
    atom = synth.caii_like_atom(7)
    atm = synth.atmos_stratified(nx=6, ny=5, nz=7, dx=90 * synth.KM, seed=9)
    serial = Level(atom, atm)
    n = zero_radiation(serial)
    js, os_ = formal_solution(serial, n)
    lev = Level(atom, atm)
    assert np.allclose(pooled_norm(lev, 3), serial.norm(), rtol=1e-14, atol=0)
    jp, op = pooled_formal_solution(lev, n)
    assert np.allclose(jp, js, rtol=1e-13, atol=0) and np.allclose(op, os_, rtol=1e-13, atol=0)
