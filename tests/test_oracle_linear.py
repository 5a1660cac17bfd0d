"""Linear-theory pin (Sec. 4): for Zel'dovich displacements at low k,
theta_p ~ delta and p ~ v with |v(k)| = Haf |delta(k)| / k, so per mode
P_tt ~ P_dt ~ P_dd and P_pp k^2 / Haf^2 ~ P_dd.  An incommensurate lattice
(n_l = 50 on a 64^3 grid) keeps the lattice comb's aliases away from the
lowest shells; lattices carry no Poisson noise, so no shot noise is
subtracted.  The mode sums below weight P_pp by each mode's own k^2."""
import numpy as np

import oracle
from synth import catalogs


def test_linear_limit_low_k():
    box, haf = 1000.0, 50.0
    pos, vel = catalogs.zeldovich(50, box, 4.0, haf=haf, seed=31)
    s = oracle.estimate(pos, vel, box=box, n_grid=64, haf=haf,
                        flags=oracle.FLAG_NO_SHOTNOISE, keep_modes=True)
    q = s.extra["modes"]
    for lo, hi in [(1, 2), (2, 3), (3, 5), (5, 8)]:
        sel = (q["n2"] >= lo * lo) & (q["n2"] < hi * hi)
        dd = np.mean(q["p_dd"][sel])
        assert abs(np.mean(q["p_tt"][sel]) / dd - 1) < 0.03
        assert abs(np.mean(q["p_dt"][sel]) / dd - 1) < 0.03
        assert abs(np.mean(q["p_pp"][sel] * q["kmag"][sel] ** 2) / haf ** 2 / dd - 1) < 0.03
