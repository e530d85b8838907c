"""The HIP path's generated Marching Cubes table against the oracle's run-time rule.

The two implement the triangulation rule independently (Python generator for
the GPU table, C function in the oracle); both must give the same ordered
triangles for all 256 cases."""
import os
import re

import numpy as np

from oracle import native
from paper_2609_20964_amd import gen_mc_table


def test_generated_table_equals_oracle_rule_all_cases():
    for case in range(256):
        gpu = np.array(gen_mc_table.case_triangles(case), dtype=np.int64).reshape(-1, 3)
        ref = native.mc_case(case).astype(np.int64)
        assert gpu.shape == ref.shape and (gpu == ref).all(), case


def test_committed_table_is_current():
    path = os.path.join(os.path.dirname(gen_mc_table.__file__), "csrc", "mc_table.inc")
    assert open(path).read() == gen_mc_table.render()
