"""Host logic of the launch-shape cache: bucketed keys, nearest-bucket lookup
within a profile, and that a workload without a cached shape runs with the
defaults rather than whatever the previous workload installed."""
import json

from paper_2601_00551_amd import autotune


class FakeCtx:
    def __init__(self):
        self.tuning = dict(autotune.DEFAULTS)


class M:
    def __init__(self, profile, directivity=1, T=4096, sampling=0):
        self.profile, self.directivity, self.T, self.sampling = profile, directivity, T, sampling


def write_cache(tmp_path, entries):
    p = tmp_path / "tuning.json"
    p.write_text(json.dumps(entries))
    return str(p)


def test_exact_and_nearest_bucket(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "_arch", lambda: "gfx950")
    a = dict(autotune.DEFAULTS, fwd_dets=1, adj_dets=2)
    b = dict(autotune.DEFAULTS, fwd_dets=8, adj_dets=8)
    path = write_cache(tmp_path, {"gfx950|p1d1|D1024|T4096|B2097152": a,
                                  "gfx950|p1d1|D512|T2048|B262144": b})
    ctx = FakeCtx()
    assert autotune.apply_cached(ctx, path, M(1), 1024, 2_000_000) == a          # exact bucket
    assert autotune.apply_cached(ctx, path, M(1, T=2048), 512, 200_000) == b     # nearest bucket
    assert autotune.apply_cached(ctx, path, M(1), 1000, 1_900_000) == a


def test_missing_profile_falls_back_to_defaults(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "_arch", lambda: "gfx950")
    tuned = dict(autotune.DEFAULTS, fwd_dets=8, adj_dets=8, adj_tile=2048)
    path = write_cache(tmp_path, {"gfx950|p1d1|D512|T2048|B262144": tuned})
    ctx = FakeCtx()
    autotune.apply_cached(ctx, path, M(1, T=2048), 512, 200_000)
    assert ctx.tuning == tuned
    # UNIFORM has no entry: the previous workload's shape must not leak through
    assert autotune.apply_cached(ctx, path, M(0), 1024, 2_000_000) == autotune.DEFAULTS


def test_point_sampling_has_its_own_buckets(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "_arch", lambda: "gfx950")
    assert autotune.shape_key("gfx950", M(1), 1024, 2_000_000) == "gfx950|p1d1|D1024|T4096|B2097152"
    assert autotune.shape_key("gfx950", M(1, sampling=1), 1024, 2_000_000) == "gfx950|p1d1s1|D1024|T4096|B2097152"
    binned = dict(autotune.DEFAULTS, fwd_dets=1, adj_dets=2)
    point = dict(autotune.DEFAULTS, fwd_dets=2, adj_dets=4)
    path = write_cache(tmp_path, {"gfx950|p1d1|D1024|T4096|B2097152": binned})
    ctx = FakeCtx()
    assert autotune.apply_cached(ctx, path, M(1), 1024, 2_000_000) == binned
    # no point-sampling entry: defaults, not the bin-mean shape
    assert autotune.apply_cached(ctx, path, M(1, sampling=1), 1024, 2_000_000) == autotune.DEFAULTS
    path = write_cache(tmp_path, {"gfx950|p1d1|D1024|T4096|B2097152": binned,
                                  "gfx950|p1d1s1|D512|T2048|B262144": point})
    assert autotune.apply_cached(ctx, path, M(1, sampling=1), 1024, 2_000_000) == point   # nearest
    assert autotune.apply_cached(ctx, path, M(1), 512, 200_000) == binned


def test_cache_file_is_reread_after_it_changes(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "_arch", lambda: "gfx950")
    a = dict(autotune.DEFAULTS, fwd_dets=1)
    b = dict(autotune.DEFAULTS, fwd_dets=8, adj_dets=8)
    path = write_cache(tmp_path, {"gfx950|p1d1|D1024|T4096|B2097152": a})
    ctx = FakeCtx()
    assert autotune.apply_cached(ctx, path, M(1), 1024, 2_000_000) == a
    assert autotune.load(path) is autotune.load(path)            # parsed once per version
    path = write_cache(tmp_path, {"gfx950|p1d1|D1024|T4096|B2097152": b, "gfx950|p0d1|D8|T8|B8": a})
    assert autotune.apply_cached(ctx, path, M(1), 1024, 2_000_000) == b
