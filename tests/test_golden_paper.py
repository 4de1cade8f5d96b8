"""Values the paper prints for a worked example (no GPU)."""
import json
import os

import numpy as np

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_vogel_spiral_array_radii_match_the_paper():
    g = json.load(open(os.path.join(GOLDEN, "vogel_array_radii.json")))
    for n, radius in g["array_radius_um"].items():
        c = W.vogel_centers(int(n), g["sphere_radius_um"])
        outer = np.max(np.hypot(c[:, 0], c[:, 1]))
        assert abs(outer - radius) <= g["printed_precision_um"]
