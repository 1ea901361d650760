"""Algorithm 2 cell behaviour on the GPU against the oracle: the Brownian
step, apoptosis (removal of cells of at least the minimum age with the death
probability, compacted out of the state in parallel, Sec 5.3.2) and the
division probability, with the Table 4.2 parameters (2,000-cell column)."""
import numpy as np
import pytest

from paper_2503_10796_amd import inputs
from tests import helpers as H

pytestmark = pytest.mark.gpu

# Table 4.2, 2,000 cells/well: growth 42 um^3 per iteration, minimum age to
# apoptosis 87, division probability 0.0215, death probability 0.033,
# maximum cell speed 1.0 um per iteration (the displacement cap), adherence
# 1.8, random movement 0.005 um per iteration
TABLE_4_2 = dict(brownian_rate=0.005, death_prob=0.033, division_prob=0.0215, min_age=87, max_disp=1.0,
                 adherence=1.8)


@pytest.fixture(scope="module")
def abm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_10796_amd import abm as _abm
    _abm.lib()
    return _abm


def spheroid_t42(n=2000, seed=21):
    """n cells in a ball of 50 (n / 1000)^(1/3) um, diameter 8 um, growth
    rates lognormal around 42 um^3 per iteration, ages uniform in [0, 100)."""
    pos, diam, vol, growth = inputs.spheroid(n, seed=seed, growth_mean=42.0)
    age = np.random.default_rng(seed + 1).integers(0, 100, size=n).astype(np.int32)
    return pos, diam, vol, growth, age


def _check_step(abm, b, st, op, cap, it):
    nu = int(st["uid"].max()) + 1
    o = H.oracle_from_state(st, op, cap=cap, next_uid=nu, iteration=it)
    b.step(1)
    o.step(1)
    ug = b.query(abm.UID)
    og, oo = np.argsort(ug), np.argsort(o.uid[: o.n])
    assert np.array_equal(ug[og], o.uid[: o.n][oo]), f"agent sets differ at iteration {it}"
    for f, ref in ((abm.VOL, o.vol), (abm.DIAM, o.diam), (abm.AGE, o.age)):
        assert np.array_equal(b.query(f)[og], ref[: o.n][oo]), (f, it)
    return o


@pytest.mark.parametrize("record", [False, True])
def test_table_4_2_spheroid_matches_the_oracle(abm, record):
    """30 iterations, each stepped once by the oracle from the GPU state:
    the same cells removed and divided (uids), the same ages, volumes and
    diameters bit for bit, positions (Brownian step bit for bit plus the
    mechanics) within the force tolerance; with recorded fields, forces
    and counts agent by agent."""
    pos, diam, vol, growth, age = spheroid_t42()
    vdiv = inputs.division_volume(12.0)
    cap = 8192
    gp = H.gpu_params(abm, box_len=0.0, div_vol=vdiv, seed=6, record=record, resort_every=10, **TABLE_4_2)
    op = H.oracle_params(box_len=0.0, div_vol=vdiv, seed=6, **TABLE_4_2)
    b = abm.Population(gp, pos, diam, vol=vol, growth=growth, capacity=cap, box_capacity=1 << 16)
    b.restore(age=age)
    removed = divided = 0
    for it in range(30):
        st = H.gpu_state(abm, b)
        o = _check_step(abm, b, st, op, cap, it)
        removed += o.n_removed
        divided += int(o.is_new[: o.n].sum())
        if record and (it + 1) % 10:
            res = H.compare_single_step(abm, b, o, check_static=False, check_nbr=False)
        else:
            res = H.compare_positions_single_step(abm, b, o, st)
        if it % 10 == 0 or it == 29:
            print(f"iteration {it}: {o.n} agents, removed so far {removed}, divided {divided}, {res}", flush=True)
    assert removed > 50 and divided > 0


def test_removals_are_deterministic_and_keep_static_agents(abm):
    """Removals on a mostly static lattice (no Brownian step): two runs are
    bitwise equal, static detection on and off give the same states (a
    removal ends no static state, Sec 5.5 condition iv), and every
    iteration matches the oracle's static flags and survivors."""
    pos, diam = inputs.relaxed_lattice(16, seed=2)
    n = pos.shape[0]
    age = np.random.default_rng(5).integers(80, 100, size=n).astype(np.int32)
    kw = dict(death_prob=0.05, min_age=87, seed=4)
    runs = []
    for det in (True, True, False):
        p = abm.Population(H.gpu_params(abm, detect_static=det, resort_every=4, **kw), pos, diam, capacity=n,
                           box_capacity=1 << 16)
        p.restore(age=age)
        runs.append(p)
    op = H.oracle_params(detect_static=True, **kw)
    for it in range(12):
        st = H.gpu_state(abm, runs[0])
        o = _check_step(abm, runs[0], st, op, n, it)
        H.compare_positions_single_step(abm, runs[0], o, st)
        gs = runs[0].query(abm.STATIC)[np.argsort(runs[0].query(abm.UID))]
        assert np.array_equal(gs, o.is_static[: o.n][np.argsort(o.uid[: o.n])]), it
        runs[1].step(1)
        runs[2].step(1)
    ref = runs[0]
    u0 = ref.query(abm.UID)
    assert u0.size < n - 100
    for other in runs[1:]:
        u = other.query(abm.UID)
        assert np.array_equal(np.sort(u), np.sort(u0))
        assert np.array_equal(other.query(abm.POS)[np.argsort(u)], ref.query(abm.POS)[np.argsort(u0)])
    assert ref.query(abm.STATIC).mean() > 0.8


def test_static_detection_with_brownian_motion_is_refused(abm):
    pos, diam = inputs.plain(64, 60.0, seed=3)
    with pytest.raises(abm.AbmError) as e:
        abm.Population(H.gpu_params(abm, detect_static=True, brownian_rate=0.01), pos, diam)
    assert e.value.code == abm.ERR_ARG
