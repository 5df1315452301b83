"""The light-cone patch used by the sampled full-size parity checks reproduces the oracle's
full-lattice result at the patch centre (CPU only)."""
import numpy as np

import workloads as WL
from parity_util import oracle_for, patch_workload


def test_patch_centre_matches_full_lattice(oracle_mod):
    w = WL.random_state(20, 18, 16, 2, seed=9, dn=0.05, du=0.03, tau_visc=0.9, tau_drag=0.56)
    k = 4
    full = oracle_for(oracle_mod, w)
    full.step(k)
    fs = [full.populations(s) for s in range(2)]
    for centre in [(0, 0, 0), (7, 3, 19), (15, 17, 10)]:
        pw, h = patch_workload(w, centre, k)
        o = oracle_for(oracle_mod, pw)
        o.step(k)
        for s in range(2):
            got = o.populations(s)[:, h, h, h]
            want = fs[s][:, centre[0], centre[1], centre[2]]
            np.testing.assert_array_equal(got, want)
