"""The incremental session (sphere insertion with dirty-block re-clipping, one captured graph per round) through the
C ABI: after any number of rounds its state equals, bit for bit, a from-scratch build with the session's sites, and
on a small case it matches the oracle."""
import numpy as np
import pytest

from paper_2403_18761_amd import synth
from tests.gpu_util import ELEMENT_ARRAYS, assert_parity, extract, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(a, dt=None):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt or torch.float32, device="cuda:0")


def _mesh(prob):
    import torch

    from paper_2403_18761_amd import rpd

    return rpd.Mesh(_dev(prob.vx), _dev(prob.vy), _dev(prob.vz), _dev(prob.tv.reshape(-1), torch.int32))


def _rebuild(mesh, sites, slots=0):
    from paper_2403_18761_amd import rpd

    s = tuple(_dev(sites[:, k]) for k in range(4))
    res = rpd.build([mesh], [s], slots=slots, block=64 if slots else 0)
    out = extract(res, 0)
    out["stats"] = res.stats()
    return out


def _same(a, b, label):
    for k in ELEMENT_ARRAYS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=f"{label}: {k}")
    assert a["stats"]["n_pairs"] == b["stats"]["n_pairs"], label


def test_session_equals_rebuild():
    from paper_2403_18761_amd import rpd

    prob, table = synth.repair_problem(N=64, n_sites=100, seed=5)
    log(f"case: session repair N64 n100 tets {prob.n_tets}")
    mesh = _mesh(prob)
    sess = rpd.Session(mesh, (_dev(prob.sx), _dev(prob.sy), _dev(prob.sz), _dev(prob.sr)),
                       tuple(_dev(x) for x in table), max_sites=100 + 6 * 32, max_insert=32)
    r0 = sess.result()
    first = extract(r0, 0)
    first["stats"] = r0.stats()
    _same(first, _rebuild(mesh, sess.sites()), "initial state")
    for rounds in (1, 2, 3):
        sess.run(rounds)
        info = sess.info()
        log("after", info["rounds"], "rounds:", info)
        res = sess.result()
        cur = extract(res, 0)
        cur["stats"] = res.stats()
        _same(cur, _rebuild(mesh, sess.sites()), f"after {info['rounds']} rounds")
    assert info["n_inserted"] > 0
    assert info["n_sites"] == 100 + info["n_inserted"]
    assert info["n_dirty_blocks"] < info["n_blocks"] * info["rounds"]


@pytest.mark.parametrize("slots", [16, 12])
def test_session_dense_sites_equals_rebuild(slots):
    """Dense sites, where workgroup site lists overflow and tets are taken one at a time with their own candidates:
    a tet's path depends on its own candidates only, so the rounds' removals take back exactly what was added and
    the state stays equal to a rebuild bit for bit (volumes included), with either vertex-slot layout of the fast
    kernel (12 slots: many more pieces redone with 64 slots, inside the kernel)."""
    from paper_2403_18761_amd import rpd

    prob = synth.torus_inside(16, 4000, 3)  # about 5 sites per tet; 6 cells violate the topology constraints
    table = synth.centroid_table(prob, 0.03)
    log(f"case: session dense torus N16 n4000 tets {prob.n_tets}")
    mesh = _mesh(prob)
    st = _rebuild(mesh, np.stack([prob.sx, prob.sy, prob.sz, prob.sr], axis=1), slots)["stats"]
    log("initial build: split", st["n_split"], "deferred", st["n_defer_block"], st["n_defer_kmax"], "big", st["n_big"])
    assert st["n_split"] > 0
    sess = rpd.Session(mesh, (_dev(prob.sx), _dev(prob.sy), _dev(prob.sz), _dev(prob.sr)),
                       tuple(_dev(x) for x in table), max_sites=4000 + 4 * 64, max_insert=64, block=64, slots=slots)
    for rounds in (1, 2, 3):
        sess.run(1)
        info = sess.info()
        res = sess.result()
        cur = extract(res, 0)
        cur["stats"] = res.stats()
        _same(cur, _rebuild(mesh, sess.sites(), slots), f"dense torus after {info['rounds']} rounds")
    log("session", info)
    assert info["n_inserted"] > 0


@pytest.mark.parametrize("rounds", [1, 4])
def test_session_matches_oracle(rounds):
    """The oracle runs the same insertion loop on its own results (oracle.repair): the session inserts the same
    sites in the same order, and its state after the rounds equals the oracle's RPD of the final sites."""
    import oracle
    from oracle import repair

    from paper_2403_18761_amd import rpd

    oracle.build(force=False)
    prob = synth.torus_inside(32, 60, 17)
    table = synth.centroid_table(prob, 0.03)
    log(f"case: session torus N32 n60 tets {prob.n_tets}, {rounds} rounds")
    want_sites, history, ref = repair.repair_loop(prob, table, rounds, max_insert=8, max_sites=60 + 40)
    assert sum(a for _, a in history) > 0
    mesh = _mesh(prob)
    sess = rpd.Session(mesh, (prob.sx, prob.sy, prob.sz, prob.sr), table, max_sites=60 + 40, max_insert=8)
    sess.run(rounds)
    info = sess.info()
    log("session", info, "oracle rounds", history)
    np.testing.assert_array_equal(sess.sites(), want_sites)
    res = sess.result()
    g = extract(res, 0)
    g["stats"] = res.stats()
    g["radii"] = want_sites[:, 3].astype(np.float64)
    assert_parity(g, ref, label="session vs oracle")


def test_session_waits_for_pending_site_writes():
    """Sites written by GPU work that is still queued on the null (default) stream when the session is created: the
    session computes on a non-blocking stream of its own, so it must wait for the caller's stream (NULL: the null
    stream) before it reads them."""
    import torch

    from paper_2403_18761_amd import rpd

    prob = synth.torus_core(16, 64, 1)
    table = synth.centroid_table(prob, 0.02)
    log(f"case: session on freshly written sites, tets {prob.n_tets}")
    mesh = _mesh(prob)
    base = [_dev(x) for x in (prob.sx, prob.sy, prob.sz, prob.sr)]
    torch.cuda.synchronize()
    busy = torch.ones(1 << 24, device="cuda:0")
    for _ in range(40):  # a queue of default-stream work ahead of the kernels that write the sites
        busy = busy * 1.0000001
    sites = tuple((b * 2.0) * 0.5 for b in base)  # exact, written by kernels behind that queue
    sess = rpd.Session(mesh, sites, tuple(_dev(x) for x in table), max_sites=64 + 16, max_insert=8)
    res = sess.result()
    got = extract(res, 0)
    got["stats"] = res.stats()
    np.testing.assert_array_equal(sess.sites(), np.stack([prob.sx, prob.sy, prob.sz, prob.sr], axis=1))
    _same(got, _rebuild(mesh, sess.sites()), "fresh sites")


def test_session_rejects_bad_arguments():
    from paper_2403_18761_amd import rpd

    prob = synth.torus_core(16, 64, 1)
    mesh = _mesh(prob)
    table = synth.centroid_table(prob, 0.02)
    sites = (prob.sx, prob.sy, prob.sz, prob.sr)
    with pytest.raises(rpd.RPDError) as e:
        rpd.Session(mesh, sites, tuple(x[:-1] for x in table), max_sites=100)
    assert e.value.code == -1
    with pytest.raises(rpd.RPDError) as e:
        rpd.Session(mesh, sites, table, max_sites=10)
    assert e.value.code == -1
    bad = list(table)
    bad[0] = bad[0].copy()
    bad[0][3] = 0.1  # off the 2^-20 grid
    with pytest.raises(rpd.RPDError) as e:
        rpd.Session(mesh, sites, tuple(bad), max_sites=100)
    assert e.value.code == -1


def _inserted_are_shrunk_spheres(prob, s, n0):
    """Every inserted site is the shrunk sphere (rounded to the grid) of one of the mesh's surface triangles."""
    from paper_2403_18761_amd import rpd

    tri, n, cen, _, _ = synth.surface_pins(prob)
    sph = rpd.shrink_spheres(tri, cen, n, np.arange(len(tri), dtype=np.int32)).astype(np.float64)
    new = s[n0:].astype(np.float64)
    assert len(new) > 0
    for q in new:
        d = np.abs(sph[:, :3] - q[:3]).max(axis=1)
        k = int(np.argmin(d))
        assert d[k] <= 4 * 2.0 ** -20 and abs(sph[k, 3] - q[3]) <= 4 * 2.0 ** -20, (q, sph[k])


def test_shrink_insertion_equals_rebuild():
    from paper_2403_18761_amd import rpd

    prob, _ = synth.repair_problem(N=64, n_sites=100, seed=5)
    log(f"case: shrink-insertion session N64 n100 tets {prob.n_tets}")
    mesh = _mesh(prob)
    sess = rpd.Session(mesh, (_dev(prob.sx), _dev(prob.sy), _dev(prob.sz), _dev(prob.sr)), None,
                       max_sites=100 + 6 * 32, max_insert=32, insertion=rpd.RPD_INSERT_SHRINK)
    for rounds in (1, 2, 3):
        sess.run(rounds)
        info = sess.info()
        log("after", info["rounds"], "rounds:", info)
        res = sess.result()
        cur = extract(res, 0)
        cur["stats"] = res.stats()
        _same(cur, _rebuild(mesh, sess.sites()), f"after {info['rounds']} rounds")
    assert info["n_inserted"] > 0
    _inserted_are_shrunk_spheres(prob, sess.sites(), 100)


def test_shrink_insertion_matches_oracle():
    import oracle

    from paper_2403_18761_amd import rpd

    oracle.build(force=False)
    prob = synth.torus_inside(32, 60, 17)
    log(f"case: shrink-insertion session torus N32 n60 tets {prob.n_tets}")
    mesh = _mesh(prob)
    sess = rpd.Session(mesh, (prob.sx, prob.sy, prob.sz, prob.sr), None, max_sites=60 + 40, max_insert=8,
                       insertion=rpd.RPD_INSERT_SHRINK)
    sess.run(3)
    info = sess.info()
    log("session", info)
    s = sess.sites()
    _inserted_are_shrunk_spheres(prob, s, 60)
    ref = oracle.rpd(prob.with_sites(s[:, 0], s[:, 1], s[:, 2], s[:, 3]), assemble=False)
    res = sess.result()
    g = extract(res, 0)
    g["stats"] = res.stats()
    assert_parity(g, ref, label="shrink session vs oracle")


def test_session_insertion_mode_arguments():
    from paper_2403_18761_amd import rpd

    prob = synth.torus_core(16, 64, 1)
    mesh = _mesh(prob)
    sites = (prob.sx, prob.sy, prob.sz, prob.sr)
    with pytest.raises(rpd.RPDError) as e:
        rpd.Session(mesh, sites, None, max_sites=100)  # the table mode needs a table
    assert e.value.code == -1
    with pytest.raises(rpd.RPDError) as e:
        rpd.Session(mesh, sites, None, max_sites=100, insertion=7)
    assert e.value.code == -1
