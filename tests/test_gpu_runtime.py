"""Runtime behaviour of the library's objects on the GPU: handles, batches and
nets give back all the device memory they take, and two handles used at the
same time on two streams give the results they give one after the other."""
import numpy as np
import pytest

from synth import make_pair, pair_seed
from synth.stereo import sensor_like

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nat():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_11924_amd.native as n
    return n


def free_bytes():
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()  # torch's own cached blocks are not the library's
    return torch.cuda.mem_get_info()[0]


def test_create_destroy_loop_returns_device_memory(nat):
    """40 rounds of create / use / destroy of a sensor-size handle (about 1 GB of
    scratch), a batch and a net: the device's free memory ends where it began
    (the HIP allocator may keep a few MB of its own)."""
    import torch
    cfg = sensor_like(1280, 720, 128)
    L = torch.randint(0, 256, (720, 1280), dtype=torch.uint8, device="cuda")
    R = torch.randint(0, 256, (720, 1280), dtype=torch.uint8, device="cuda")
    out = [torch.empty((720, 1280), dtype=torch.float32, device="cuda") for _ in range(2)] + \
          [torch.empty((720, 1280), dtype=torch.uint8, device="cuda")]
    small = sensor_like(160, 96, 64)["params"]
    # one round first, so that lazily loaded code objects are resident
    ss = nat.SimSense(cfg["params"])
    ss.compute(L, R, *out)
    ss.close()
    before = free_bytes()
    for i in range(40):
        ss = nat.SimSense(cfg["params"])
        if i % 10 == 0:
            ss.compute(L, R, *out)
        ss.close()
        b = nat.Batch([small, small])
        b.close()
        net = nat.Net(4096, seed=i)
        net.close()
    after = free_bytes()
    assert before - after <= 16 << 20, (before, after)


def test_two_handles_on_two_streams_match_sequential(orc, nat):
    """A 1280x720 8-path handle and a 640x480 4-path handle, each on its own
    stream, both enqueued before either is waited for, several times over: every
    output equals the handle's result computed alone."""
    import torch
    cfg_a, cfg_b = sensor_like(1280, 720, 128), sensor_like(640, 480, 96)
    pa = cfg_a["params"]
    pb = dict(cfg_b["params"], num_paths=4)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ins = []
    for cfg, k in ((cfg_a, 0), (cfg_b, 1)):
        pr = make_pair(cfg["spec"], pair_seed(6, 400 + k))
        ins.append((t(orc.ir_noise(pr.left, pr.gamma_l, pr.n_l)), t(orc.ir_noise(pr.right, pr.gamma_r, pr.n_r))))
    ha, hb = nat.SimSense(pa), nat.SimSense(pb)
    ref_a = [x.cpu().numpy() for x in ha(*ins[0])]
    ref_b = [x.cpu().numpy() for x in hb(*ins[1])]
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(sa):
            oa = [torch.empty((720, 1280), dtype=torch.float32, device="cuda") for _ in range(2)] + \
                 [torch.empty((720, 1280), dtype=torch.uint8, device="cuda")]
            ha.compute(*ins[0], *oa, stream=sa)
        with torch.cuda.stream(sb):
            ob = [torch.empty((480, 640), dtype=torch.float32, device="cuda") for _ in range(2)] + \
                 [torch.empty((480, 640), dtype=torch.uint8, device="cuda")]
            hb.compute(*ins[1], *ob, stream=sb)
        torch.cuda.synchronize()
        for got, want in zip(oa, ref_a):
            assert np.array_equal(got.cpu().numpy(), want), rep
        for got, want in zip(ob, ref_b):
            assert np.array_equal(got.cpu().numpy(), want), rep
    ha.close()
    hb.close()
