"""Small seeded problems shared by the tests (built from the generator)."""
import functools
import math

import numpy as np

from paper_1611_07289_amd import synth


def brute_problem(seed: int = 7, rot_deg: float = 8.0, trans: float = 0.7) -> synth.Problem:
    """8^3 volume, 3 orthogonal stacks of 8x8x2 (thickness 4), 4x4 patches with
    stride 2: M = 3 * 2 * 9 = 54 patches, 864 samples."""
    g = synth.iso_grid(8)
    x = np.random.default_rng(seed).uniform(0, 1000, size=(8, 8, 8)).astype(np.float32)
    c = synth.grid_center(g)
    stacks = [synth.make_stack(c, *fr, 8, 8, 2, (1, 1), 4.0, (1.0, 1.0, 4.0))
              for fr in synth.orthogonal_frames()]
    P = synth.square_patches(stacks, 4, 2)
    th = synth.random_motion(P.M, rot_deg, trans, seed + 1)
    return synth.Problem("brute8", g, stacks, P, x, th, np.zeros(P.M, bool), seed)


@functools.lru_cache(maxsize=None)
def tiny():
    return synth.tiny_problem()
