"""GPU parity of the pair potential (truncated Lennard-Jones over the
Tersoff context's device list, the paper's Algorithm 1) against the FP64
oracle, through the C ABI.

Bars: FP64 <= 1e-12 (energy, norm-wise forces, virial).  Mixed (FP32 V and
dV/dr from the FP64 squared distance rounded to FP32, FP64 accumulation):
(sigma/r)^12 carries 12 roundings of ~6e-8, so a pair term is good to
~1e-6 relative; the bars are 1e-6 on the energy relative to sum |V|, 1e-5
norm-wise on forces and virial."""
import numpy as np
import pytest
import torch

from oracle import pair
from paper_1607_02904_amd import inputs

pytestmark = pytest.mark.gpu

EPS, SIG, RC = 0.05, 2.1, 3.0  # minimum at 2.36 A, the Si bond length


@pytest.fixture(scope="module")
def model():
    from paper_1607_02904_amd.tersoff import Tersoff, table_element
    m = Tersoff(table_element("Si(B)"))  # list radius: the Tersoff cutoff + skin
    yield m
    m.close()


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    d = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (d if d > 0 else 1.0)


def _run(model, x, t, box, precision, skin):
    xd = torch.as_tensor(x, device="cuda")
    td = torch.as_tensor(t, device="cuda")
    model.build_nlist(xd, td, box, skin)
    o = model.pair_compute(xd, box, EPS, SIG, RC, precision)
    torch.cuda.synchronize()
    model.sync()
    return float(o["energy"].item()), o["forces"].cpu().numpy(), o["virial"].cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("skin", [0.0, 0.5])
def test_pair_matches_oracle(model, precision, skin):
    x, t, box = inputs.si_bulk(ncell=4, sigma=0.15, seed=31)
    e, f, w = _run(model, x, t, box, precision, skin)
    er, fr, wr = pair.lj_compute(x, box, EPS, SIG, RC)
    if precision == 0:
        assert abs(e - er) <= 1e-12 * abs(er)
        assert _rel(f, fr) <= 1e-12
        assert _rel(w, wr) <= 1e-12
    else:
        scale = 0.5 * np.sum(np.abs(_pair_energies(x, box)))
        assert abs(e - er) <= 1e-6 * scale, (e, er)
        assert _rel(f, fr) <= 1e-5
        assert _rel(w, wr) <= 1e-5
    assert np.abs(f.sum(axis=0)).max() <= 1e-9


def _pair_energies(x, box):
    """Per-atom sums of |V| (the conditioning scale of the energy sum)."""
    out = np.zeros(len(x))
    for i in range(len(x)):
        d = x - x[i]
        d -= box * np.round(d / box)
        r = np.sqrt(np.sum(d * d, axis=1))
        m = (r > 0) & (r < RC)
        v, _ = pair.lj_pair(r[m], EPS, SIG)
        out[i] = np.sum(np.abs(v))
    return out


def test_pair_cutoff_beyond_the_list_is_refused(model):
    from paper_1607_02904_amd.tersoff import TersoffError
    x, t, box = inputs.si_small()
    xd = torch.as_tensor(x, device="cuda")
    model.build_nlist(xd, torch.as_tensor(t, device="cuda"), box, 0.5)
    with pytest.raises(TersoffError) as ei:
        model.pair_compute(xd, box, EPS, SIG, 3.6)  # beyond the Tersoff cutoff (3.0 or 3.2 A)
    assert ei.value.name == "TERS_ERR_INVALID_ARG"


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_pair_full_size(model, precision):
    """The benchmark's pair-potential evaluation: 512,000-atom Si over the
    list of skin 0.5, against the oracle with its pairs enumerated by a k-d
    tree (every atom's force, the energy and the virial)."""
    x, t, box = inputs.si_bulk(40)
    e, f, w = _run(model, x, t, box, precision, 0.5)
    er, fr, wr = pair.lj_compute_pairs(x, box, EPS, SIG, RC)
    if precision == 0:
        assert abs(e - er) <= 1e-12 * abs(er)
        assert _rel(f, fr) <= 1e-12
        assert _rel(w, wr) <= 1e-12
    else:
        assert abs(e - er) <= 1e-6 * abs(er), (e, er)
        assert _rel(f, fr) <= 1e-5
        assert _rel(w, wr) <= 1e-5

