"""Pins the reading of the time-reduction column of Table 1 (section 4.2):
reduction = (T_1 - T_m) / T_1 * 100 per platform (the printed formula is garbled)."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def time_reduction(t1, tm):
    return (t1 - tm) / t1 * 100.0


def test_table1_reduction_reading():
    tab = np.loadtxt(os.path.join(HERE, "golden", "table1_total_time.txt"))
    r1, m1 = tab[0, 1], tab[0, 3]
    for row in tab[1:]:
        assert abs(time_reduction(r1, row[1]) - row[2]) <= 0.011
        assert abs(time_reduction(m1, row[3]) - row[4]) <= 0.011
