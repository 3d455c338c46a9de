"""The allocation-free start, pflb_init_fields_noalloc, through the C ABI: the state it
loads equals the one pflb_init_fields loads with a caller work buffer, bit for bit, on
calls in a row whose domains shrink (the library's fixed array keeps the previous
call's contents), in both storages; a domain above the array's limit is refused with
PFLB_ERR_PARAM and leaves the context's state unchanged."""
import numpy as np
import pytest
import torch

import pfinputs

pytestmark = pytest.mark.gpu


def _pair(cfg, storage):
    from paper_1812_00118_amd import Sim
    phi, u, P = pfinputs.fields(cfg)
    a = Sim(cfg, storage=storage)
    a.init_fields(phi, u, P)
    b = Sim(cfg, storage=storage)
    b.init_fields_noalloc(phi, u, P)
    ha, ga = a.get_state()
    hb, gb = b.get_state()
    torch.cuda.synchronize()
    assert torch.equal(ha, hb) and torch.equal(ga, gb), cfg["name"]
    # and the states evolve identically
    a.step(3)
    b.step(3)
    ra, rb = a.read(), b.read()
    for k in ra:
        assert torch.equal(ra[k], rb[k]), (cfg["name"], k)
    return a.N


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_noalloc_start_matches_work_buffer_start(storage):
    from paper_1812_00118_amd._lib import lib
    limit = lib().pflb_noalloc_scratch_bytes()
    assert limit == 64 * 1024 * 1024
    big = pfinputs.rising_bubble(n=48, R=10.0)            # 110,592 sites, 16.8 MB staged
    small = pfinputs.rising_bubble(n=20, R=5.0)           # 8,000 sites
    d2 = pfinputs.static_droplet(n=40, R=10.0)            # 1,600 D2Q9 sites
    sizes = [_pair(c, storage) for c in (big, small, d2)]
    print(f"\nno-alloc start, {storage}: bitwise equal on {sizes} sites in a row")
    assert sizes[0] > sizes[1] > sizes[2]


def test_noalloc_start_refuses_domains_above_the_limit():
    from paper_1812_00118_amd import Sim
    from paper_1812_00118_amd._lib import PflbError
    # 77 x 77 x 75 = 444,675 D3Q19 sites: 2 * 19 * 4 bytes each exceed 64 MiB
    cfg = dict(pfinputs.rising_bubble(n=48, R=10.0), shape=(77, 77, 75))
    sim = Sim(cfg)
    phi, u, P = pfinputs.fields(dict(cfg))
    sim.init_fields(phi, u, P)
    h0, g0 = sim.get_state()
    with pytest.raises(PflbError) as e:
        sim.init_fields_noalloc(phi, u, P)
    assert "PFLB_ERR_PARAM" in str(e.value) and "too large" in str(e.value)
    h1, g1 = sim.get_state()
    torch.cuda.synchronize()
    assert torch.equal(h0, h1) and torch.equal(g0, g1)
