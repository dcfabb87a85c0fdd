"""Batched JTV-MAP fits (mpm_fit_batch): several volumes of different sizes,
protocols and priors run in lockstep with every kernel launch serving all of
them.  Each volume's maps, report and objective trace equal its mpm_fit alone
bit for bit, and the oracle's to the FP32 bound."""
import numpy as np
import pytest

from conftest import cuda, f32, map_errors, observations, well_posed
from paper_2102_01604_amd import _lib, synth

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _lib.load()
    return torch


def _volume(orc, dims, seed, echoes=(8, 8, 6), init="const"):
    c = synth.make_case("map_brain", dims=dims, seed=seed, echoes=echoes)
    c["b1"] = f32(c["b1"])
    x = observations(orc, c)
    opts = dict(c["opts"], n_outer=3, n_gn=3, n_cg=12)
    if init == "const":
        y0 = f32(orc.default_init(c["proto"], x.astype(np.float64), c["b1"]))
        opts.update(init="const", init_const=[float(v) for v in y0])
    return c, x, opts


def _tensors(torch, c, x):
    return cuda(x.astype(np.float32)), cuda(c["b1"].astype(np.float32)), \
        torch.zeros((4, x.shape[1]), dtype=torch.float32, device="cuda")


def test_batch_equals_fits_alone(torch_cuda, orc):
    torch = torch_cuda
    vols = [_volume(orc, (24, 20, 12), 91), _volume(orc, (70, 37, 41), 92, init="default"),
            _volume(orc, (2, 1, 1), 93), _volume(orc, (33, 9, 64), 94, echoes=(6, 6, 6)),
            _volume(orc, (64, 16, 5), 95)]
    fits, solo = [], []
    for c, x, opts in vols:
        X, B1, M = _tensors(torch, c, x)
        fits.append((c["proto"], c["dims"], X, B1, opts, M))
        M2 = torch.zeros_like(M)
        rep, tr = _lib.mpm_fit(c["proto"], c["dims"], X, B1, opts, M2)
        solo.append((M2.cpu().numpy(), rep, tr))
    print("batch of", [v[0]["dims"] for v in vols], flush=True)
    out = _lib.mpm_fit_batch(fits)
    torch.cuda.synchronize()
    for (c, x, opts), f, (y_solo, rep_solo, tr_solo), (rep, tr) in zip(vols, fits, solo, out):
        y = f[5].cpu().numpy()
        print(c["dims"], rep)
        assert np.array_equal(y, y_solo), c["dims"]
        assert rep == rep_solo
        assert np.array_equal(tr, tr_solo, equal_nan=True)
    # one volume of the batch against the oracle
    c, x, opts = vols[0]
    y_orc, rep_o, tr_o = orc.fit(c["proto"], c["dims"], x.astype(np.float64), c["b1"], opts)
    y = fits[0][5].cpu().numpy().astype(np.float64)
    rel = map_errors(y, y_orc)[0]
    print("batched volume vs oracle", rel)
    assert (rel <= TOL).all()
    fin = np.isfinite(tr_o)
    assert np.allclose(out[0][1][fin], tr_o[fin], rtol=1e-6)


def test_batch_equals_fits_alone_with_halved_steps(torch_cuda, orc):
    """Plain Gauss-Newton loading, whose full steps the acceptance test of
    Sec. 2.7 sometimes rejects: inside an outer loop a halved step is then
    taken.  A fit alone lets its full-step acceptance pass evaluate the next
    likelihood pass in advance and discards it after a halved step; a batched
    fit evaluates every pass in turn.  Both give the same bits, and the oracle's
    maps and trace."""
    torch = torch_cuda
    vols = []
    for dims, seed in [((24, 20, 12), 101), ((16, 12, 10), 102)]:
        c = synth.make_case("map_brain", dims=dims, seed=seed)
        c["b1"] = f32(c["b1"])
        x = observations(orc, c)
        y0 = f32(orc.default_init(c["proto"], x.astype(np.float64), c["b1"]))
        opts = dict(c["opts"], n_outer=3, n_gn=4, n_cg=16, loading="gn", max_halvings=4, init="const",
                    init_const=[float(v) for v in y0])
        # without halvings the oracle rejects some full steps: the case takes halved ones
        _, rep0, _ = orc.fit(c["proto"], dims, x.astype(np.float64), c["b1"], dict(opts, max_halvings=0))
        assert rep0["rejected"] > 0, dims
        vols.append((c, x, opts))
    fits, solo = [], []
    for c, x, opts in vols:
        X, B1, M = _tensors(torch, c, x)
        fits.append((c["proto"], c["dims"], X, B1, opts, M))
        M2 = torch.zeros_like(M)
        rep, tr = _lib.mpm_fit(c["proto"], c["dims"], X, B1, opts, M2)
        solo.append((M2.cpu().numpy(), rep, tr))
    out = _lib.mpm_fit_batch(fits)
    torch.cuda.synchronize()
    for (c, x, opts), f, (y_solo, rep_solo, tr_solo), (rep, tr) in zip(vols, fits, solo, out):
        y = f[5].cpu().numpy()
        print(c["dims"], rep)
        assert np.array_equal(y, y_solo), c["dims"]
        assert rep == rep_solo
        assert np.array_equal(tr, tr_solo, equal_nan=True)
        y_orc, rep_o, tr_o = orc.fit(c["proto"], c["dims"], x.astype(np.float64), c["b1"], opts)
        rel = map_errors(y.astype(np.float64), y_orc)[0]
        print("halved steps: gpu vs oracle", rel, rep_o)
        assert (rel <= TOL).all() and rep["gn_done"] == rep_o["gn_done"] == 12
        fin = np.isfinite(tr_o)
        assert np.array_equal(np.isfinite(tr), fin) and np.allclose(tr[fin], tr_o[fin], rtol=1e-5)


def test_batch_fp16_offsets_and_incompatible_schedule(torch_cuda, orc):
    torch = torch_cuda
    vols = [_volume(orc, (32, 24, 16), 96), _volume(orc, (40, 27, 19), 97)]
    fits, solo = [], []
    for c, x, opts in vols:
        X = cuda(x.astype(np.float32))
        Q = torch.empty(X.shape, dtype=torch.float16, device="cuda")
        off = _lib.mpm_pack_echoes(X, Q)
        o = dict(opts, echo_offset=off)
        B1 = cuda(c["b1"].astype(np.float32))
        M = torch.zeros((4, x.shape[1]), dtype=torch.float32, device="cuda")
        fits.append((c["proto"], c["dims"], Q, B1, o, M))
        M2 = torch.zeros_like(M)
        rep, _ = _lib.mpm_fit(c["proto"], c["dims"], Q, B1, o, M2)
        solo.append((M2.cpu().numpy(), rep))
    out = _lib.mpm_fit_batch(fits)
    for f, (y_solo, rep_solo), (rep, _) in zip(fits, solo, out):
        assert np.array_equal(f[5].cpu().numpy(), y_solo) and rep == rep_solo
    bad = list(fits)
    bad[1] = bad[1][:4] + (dict(bad[1][4], n_cg=11),) + bad[1][5:]
    with pytest.raises(_lib.MpmError) as err:
        _lib.mpm_fit_batch(bad)
    assert err.value.status == 2 and "schedule" in str(err.value)
    ml = list(fits)
    ml[0] = ml[0][:4] + (dict(ml[0][4], mode="ml"),) + ml[0][5:]
    with pytest.raises(_lib.MpmError) as err:
        _lib.mpm_fit_batch(ml)
    assert err.value.status == 2
