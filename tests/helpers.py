"""Shared test glue: turning scene inputs into oracle views and parameter rows."""
import numpy as np

import oracle
from paper_2404_06926_amd import scenes


def oview(cam: scenes.Camera) -> oracle.OView:
    return oracle.OView(cam=cam.cam16(), W=cam.width, H=cam.height,
                        E=cam.exposure.astype(np.float64), bg=cam.bg.astype(np.float64))


def gauss_row(mean, log_scale, quat=(1.0, 0.0, 0.0, 0.0), logit=0.0, dc=(0.5, 0.5, 0.5), deg=0,
              rest=None):
    """One parameter row (float64) in the layout mean, log-scale, quat, logit, SH[k][c]."""
    K = (deg + 1) ** 2
    sh = np.zeros((K, 3))
    sh[0] = dc
    if rest is not None:
        sh[1:] = rest
    ls = np.broadcast_to(np.asarray(log_scale, np.float64), (3,))
    return np.concatenate([np.asarray(mean, np.float64), ls, np.asarray(quat, np.float64),
                           [logit], sh.reshape(-1)])


def logit(p):
    return float(np.log(p / (1 - p)))


Y00 = 0.5 / np.sqrt(np.pi)  # degree-0 real spherical harmonic, 1 / (2 sqrt(pi))


def dc_for_colour(c):
    """SH DC coefficient that renders as colour c (colour = Y00 * dc + 0.5)."""
    return (np.asarray(c, np.float64) - 0.5) / Y00
