"""Obstacle geometry (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Ch. 5, "Model and Methods": every lattice node inside an impurity is a
bounce-back node.  Impurities are discs; the channel of the batched workloads
adds solid rows at the bottom and top border.
"""
import numpy as np


def disc_mask(nx, ny, discs):
    """Solid where the node (x, y) lies inside a disc: dx^2 + dy^2 <= r^2,
    with dx, dy the periodic (minimum-image) distances to the centre."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    solid = np.zeros((ny, nx), bool)
    for cx, cy, r in discs:
        dx = x - cx
        dx = dx - nx * np.round(dx / nx)
        dy = y - cy
        dy = dy - ny * np.round(dy / ny)
        solid |= dx * dx + dy * dy <= r * r
    return solid


def channel_mask(nx, ny, discs=()):
    """Walls at y = 0 and y = ny - 1 plus the discs."""
    solid = disc_mask(nx, ny, discs)
    solid[0, :] = True
    solid[-1, :] = True
    return solid
