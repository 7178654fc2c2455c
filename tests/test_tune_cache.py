"""Host logic of the kernel-variant cache (no GPU): keys depend on the
architecture, widths, box count and the kernel-selecting options only, and
stored choices round-trip through the file."""
from paper_2211_14438_amd import tune_cache as TC


def test_key_fields():
    k1 = TC.cache_key("gfx950", [6, 64, 64, 64, 4], 1024, L=2, precision="fp32", plan="learned", sched="batched",
                      pred=object(), workspace=object())
    k2 = TC.cache_key("gfx950", [6, 64, 64, 64, 4], 1024, L=2, precision="fp32", plan="learned", sched="batched")
    assert k1 == k2  # buffers and predictors do not enter
    assert k1 != TC.cache_key("gfx942", [6, 64, 64, 64, 4], 1024, L=2, precision="fp32", plan="learned",
                              sched="batched")
    assert k1 != TC.cache_key("gfx950", [6, 64, 64, 4], 1024, L=2, precision="fp32", plan="learned", sched="batched")
    assert k1 != TC.cache_key("gfx950", [6, 64, 64, 64, 4], 512, L=2, precision="fp32", plan="learned",
                              sched="batched")
    assert k1 != TC.cache_key("gfx950", [6, 64, 64, 64, 4], 1024, L=3, precision="fp32", plan="learned",
                              sched="batched")


def test_store_and_load(tmp_path):
    path = str(tmp_path / "tune.json")
    assert TC.load(path) == {}
    TC.store(path, "a", [3, 0, 1, 2], 0.95)
    TC.store(path, "b", [1, 1, 1, 1], 2.5)
    d = TC.load(path)
    assert d["a"] == {"choice": [3, 0, 1, 2], "ms_per_pass": 0.95}
    assert d["b"]["choice"] == [1, 1, 1, 1]
