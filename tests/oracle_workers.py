"""Per-shard oracle work for the full-size checks, run in spawned worker
processes (imports only NumPy and the oracle): the eq. (5) partial sums
with their derivatives along v, and the absolute sums behind the error
yardsticks S_p and SH_p, both additive over event shards."""

import numpy as np

import oracle
from oracle import pwa_oracle


def shard(args):
    data, mc, model, theta, v = args
    parts = oracle.partials(data, mc, model, theta, v=v)
    th = np.asarray(theta, dtype=np.float64)
    vv = np.asarray(v, dtype=np.float64)
    hF, gF, _ = pwa_oracle._hvp_abs_sums(data, model, th, vv, True)
    hG, gG, G = pwa_oracle._hvp_abs_sums(mc, model, th, vv, False)
    return parts, (hF, gF, hG, gG, G)
