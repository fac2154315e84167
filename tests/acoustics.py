"""Speed of the pressure pulses that leave the interface of the RTI box
(Section 4 reads the local sound speed off the slopes of the pulse peaks in
the (y, t) plane of the disturbance pressure).

``pulse_speeds`` follows the largest |p - p_h| on each side of the interface
along a vertical line: the first record picks the global peak of each half
(beyond 3 nodes from the interface), later records search a window that moves
with the previous peak; peaks are refined by a parabola through three nodes.
It returns the least-squares slopes of distance against time, upper and
lower side, in box lengths per time unit.
"""
import numpy as np


def _peak(a, lo, hi):
    lo, hi = max(lo, 1), min(hi, a.size - 1)
    i = int(np.argmax(a[lo:hi])) + lo
    den = a[i - 1] - 2.0 * a[i] + a[i + 1]
    return i + (0.5 * (a[i - 1] - a[i + 1]) / den if den != 0.0 else 0.0)


def pulse_speeds(times, lines, ny, window=0.05):
    """times: record times; lines: disturbance pressure along y (ny nodes on
    [0, 1], interface between nodes ny//2 - 1 and ny//2) at those times."""
    h = 1.0 / (ny - 1)
    j0 = ny // 2
    w = int(window / h) + 1
    pu = pl = None
    up_d, lo_d = [], []
    for line in lines:
        a = np.abs(np.asarray(line, dtype=np.float64))
        up, dn = a[j0:], a[:j0][::-1]
        pu = _peak(up, 3, up.size - 1) if pu is None else _peak(up, int(pu) - 2, int(pu) + w)
        pl = _peak(dn, 3, dn.size - 1) if pl is None else _peak(dn, int(pl) - 2, int(pl) + w)
        up_d.append((pu + 0.5) * h)
        lo_d.append((pl + 0.5) * h)
    t = np.asarray(times, dtype=np.float64)
    return float(np.polyfit(t, up_d, 1)[0]), float(np.polyfit(t, lo_d, 1)[0])
