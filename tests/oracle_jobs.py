"""Oracle runs for worker processes of the GPU tests.  This module imports
neither torch nor the library, so a spawned worker never touches the GPU."""
import numpy as np

import pbn_synth as ps
from oracle import simulate as osim


def c4_network_run(args):
    """Oracle trajectories of network k of the C4 batch:
    (k, seed, trajectory ids, steps, count_from, target sets) -> oracle.run's dict."""
    k, seed, sample, steps, count_from, target_sets = args
    net = ps.batch_c4_network(k)
    return osim.run(net, seed, np.asarray(sample), steps, count_from=count_from, targets=target_sets)
