"""Host-side logic that the GPU runs rely on, checked on the CPU."""
import numpy as np

import bench
from oracle import sim as osim
from paper_2503_10796_amd import inputs
from tests import helpers as H


def test_lineage_count_equals_the_oracle_agent_count():
    # Algorithm 2: growth and division do not depend on positions, so the
    # agent count of the scale run follows from volumes and rates alone.
    pos, diam, vol, growth = inputs.spheroid(1000, seed=3, growth_scale=8.0)
    vdiv = inputs.division_volume(12.0)
    counts = bench.lineage_counts(vol, growth, vdiv, 100)
    o = osim.OracleSim(pos, diam, H.oracle_params(box_len=0.0, div_vol=vdiv, seed=3), vol=vol, growth=growth,
                       cap=int(counts[-1]) + 16)
    seen = [o.n]
    for _ in range(100):
        o.step(1)
        seen.append(o.n)
    assert np.array_equal(np.array(seen), counts.astype(np.int64))
    assert counts[-1] > counts[0]  # divisions happen within the checked window


def test_scale_run_reaches_five_million_agents():
    pos, diam, vol, growth = inputs.spheroid(1000, seed=3, growth_scale=8.0)
    counts = bench.lineage_counts(vol, growth, inputs.division_volume(12.0), 600)
    assert 4.5e6 < counts[-1] < 5.5e6
