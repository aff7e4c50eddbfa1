"""Material files (nam_material_save / nam_material_load_file): a saved and reloaded material
decodes bit for bit as the original, with and without learned frames and in every precision;
damaged files are rejected with NAM_E_IO."""
import os

import numpy as np
import pytest

from paper_2305_02678_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def nam(torch):
    from paper_2305_02678_amd import nam as n
    n.lib()
    return n


@pytest.fixture(scope="module")
def ctx(nam):
    return nam.Context(0)


def _material(nf, address=wl.WRAP, seed=51):
    r = wl.rngs(seed)
    return wl.make_material(r[0], r[1], 64, 32, 16, 6, [64] * 3, address=address, n_frames=nf)


@pytest.mark.parametrize("nf,address", [(0, wl.WRAP), (2, wl.CLAMP), (1, wl.WRAP)])
def test_round_trip_is_bit_exact(nam, ctx, torch, tmp_path, nf, address):
    m = _material(nf, address)
    a = nam.Material.from_workload(ctx, m)
    path = str(tmp_path / "m.nam")
    a.set_precision(nam.F16)                      # the file holds the FP32 master copy regardless
    a.save(path)
    b = nam.Material.load_file(ctx, path)
    assert b.dims == m.dims and b.n_frames == nf and b.channels == 16
    assert a.footprint() > b.footprint()          # a also holds its FP16 copies
    q = wl.uniform_queries(np.random.default_rng(2), 4000, -0.5, 5.5)
    dq = nam.to_device(q)
    xi = torch.from_numpy(np.random.default_rng(3).random(4000, dtype=np.float32)).cuda()
    for prec in (nam.F32, nam.F16):
        a.set_precision(prec)
        b.set_precision(prec)
        for x in (None, xi):
            assert torch.equal(nam.decode(a, *dq, xi=x), nam.decode(b, *dq, xi=x)), (prec, x is None)
    b.save(str(tmp_path / "m2.nam"))
    assert open(path, "rb").read() == open(str(tmp_path / "m2.nam"), "rb").read()


def test_damaged_files_are_rejected(nam, ctx, tmp_path):
    a = nam.Material.from_workload(ctx, _material(2))
    path = str(tmp_path / "m.nam")
    a.save(path)
    blob = open(path, "rb").read()

    def load(data):
        p = str(tmp_path / "bad.nam")
        with open(p, "wb") as f:
            f.write(data)
        return nam.Material.load_file(ctx, p)

    flipped = bytearray(blob)
    flipped[len(blob) // 2] ^= 0x40
    for data, what in ((blob[:-9], "truncated"), (bytes(flipped), "checksum"), (b"XAMMAT01" + blob[8:], "magic"),
                       (blob[:8] + np.int32(1 << 20).tobytes() + blob[12:], "size")):
        with pytest.raises(nam.NamError, match="NAM_E_IO"):
            load(data)
    with pytest.raises(nam.NamError, match="NAM_E_IO"):
        nam.Material.load_file(ctx, str(tmp_path / "missing.nam"))
    with pytest.raises(nam.NamError, match="NAM_E_IO"):
        a.save(str(tmp_path / "no_such_dir" / "m.nam"))
    assert os.path.getsize(path) == len(blob)
