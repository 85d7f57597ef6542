"""GPU: the autotuner's persistent cache (mpdc_autotune's cache_path).  A
first call times every legal shape and stores its choice; a second state of
the same configuration takes the stored choice without timing; a stored
choice that is not legal for the state is retuned and replaced; other
configurations add lines; results are bitwise identical throughout."""
import time

import numpy as np
import pytest

from paper_2404_08849_amd.inputs import initial as ic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpdc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_08849_amd.mpdc as m
    return m


def _state(mpdc, g, s, K, policy):
    st = mpdc.State(g, mpdc.MODEL_HDC, policy, K=K, dt=600.0, sigma=ic.sigma_interfaces(K))
    st.state_write(mpdc.FIELD_PS, s["ps"][:, None])
    st.state_write(mpdc.FIELD_THETA, s["Theta"][:, :, None])
    st.state_write(mpdc.FIELD_U, s["u"][:, :, None])
    return st


def test_autotune_cache_roundtrip(mpdc, mesh_cache, tmp_path):
    m = mesh_cache(4)
    K = 10
    s = ic.hdc_jet(m, K, seed=2000)
    g = mpdc.Mesh(m)
    path = str(tmp_path / "tune.txt")
    st = _state(mpdc, g, s, K, mpdc.POLICY_MIX)
    t0 = time.perf_counter()
    shapes = st.autotune(cache_path=path)
    t_tune = time.perf_counter() - t0
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and "policy=1" in lines[0] and "K=10" in lines[0]
    st.dycore_step(3)
    ref = st.state_read(mpdc.FIELD_U)
    # a second state of the same configuration takes the stored choice, untimed
    st2 = _state(mpdc, g, s, K, mpdc.POLICY_MIX)
    t0 = time.perf_counter()
    shapes2 = st2.autotune(cache_path=path)
    t_cached = time.perf_counter() - t0
    print("tuning %.3f s, from the cache %.4f s, shapes %s" % (t_tune, t_cached, shapes), flush=True)
    assert shapes2 == shapes and t_cached < 0.25 * t_tune
    st2.dycore_step(3)
    assert np.array_equal(st2.state_read(mpdc.FIELD_U), ref)
    # another configuration adds a line; the first is kept
    st3 = _state(mpdc, g, s, K, mpdc.POLICY_DBL)
    st3.autotune(cache_path=path)
    lines = open(path).read().splitlines()
    assert len(lines) == 2 and "policy=1" in lines[0] and "policy=0" in lines[1]
    # an illegal stored choice (two values per lane in a K = 10 column needs an even count
    # of lanes; 1000 cells per work-group is over the limit) is retuned and replaced
    key, vals = lines[0].split(" | ")
    bad = key + " | " + " ".join(["1", "1000"] * 4)
    open(path, "w").write(bad + "\n" + lines[1] + "\n")
    st4 = _state(mpdc, g, s, K, mpdc.POLICY_MIX)
    st4.autotune(cache_path=path)
    lines = open(path).read().splitlines()
    assert len(lines) == 2 and bad not in lines
    st4.dycore_step(3)
    assert np.array_equal(st4.state_read(mpdc.FIELD_U), ref)
    # no cache: plain tuning, nothing written
    assert len(st4.autotune()) == 4 and len(open(path).read().splitlines()) == 2


def test_autotune_cache_unwritable_is_an_error(mpdc, mesh_cache, tmp_path):
    m = mesh_cache(2)
    K = 4
    s = ic.hdc_jet(m, K, seed=2000)
    st = _state(mpdc, mpdc.Mesh(m), s, K, mpdc.POLICY_DBL)
    with pytest.raises(mpdc.MpdcError) as e:
        st.autotune(cache_path=str(tmp_path / "no_such_dir" / "tune.txt"))
    assert e.value.code == -1 and "autotune cache" in str(e.value)


@pytest.mark.parametrize("policy", ["MIX", "DBL", "MIX_DBL_MASS"])
def test_autotune_leaves_the_state_unchanged(mpdc, mesh_cache, policy):
    """Tuning (the timed launches write only the stage scratch set, also when
    they store the FP64 state as the last stage does) changes neither the
    state nor, after it, the steps' results."""
    m = mesh_cache(4)
    K = 10
    s = ic.hdc_jet(m, K, seed=2000)
    g = mpdc.Mesh(m)
    fields = (mpdc.FIELD_PS, mpdc.FIELD_THETA, mpdc.FIELD_U)
    pol = getattr(mpdc, "POLICY_" + policy)
    st = _state(mpdc, g, s, K, pol)
    before = [st.state_read(f) for f in fields]
    st.autotune()
    after = [st.state_read(f) for f in fields]
    assert all(np.array_equal(x, y) for x, y in zip(before, after))
    ref = _state(mpdc, g, s, K, pol)
    st.dycore_step(3)
    ref.dycore_step(3)
    assert all(np.array_equal(st.state_read(f), ref.state_read(f)) for f in fields)
