"""Accuracy metric of the experiments section.

Percentage error (Sec. 6.1, eq. percentError): E = (100/N) sum_i Delta_i / R_i
over the N grid nodes, with R_i the true distance and Delta_i = |S_i - R_i|.
Reading: at a source node R_i = 0 and Delta_i vanishes with tau, so the
term is taken as 0 while N still counts every node.  With this reading the
oracle reproduces the maxima printed in Table 2 to within about 5 per cent
(the reading that drops source nodes from N gives 1.5 times the printed
values at every tau).
"""

from __future__ import annotations

import numpy as np


def percent_error(S, R):
    S = np.asarray(S, dtype=np.float64).ravel()
    R = np.asarray(R, dtype=np.float64).ravel()
    keep = R > 0
    return float(100.0 * np.sum(np.abs(S[keep] - R[keep]) / R[keep]) / len(R))
