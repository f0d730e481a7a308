"""What the trained selector gains: on held-out corpus tensors (seeds the
network never saw), every candidate of every mode is timed (exhaustive), and
the network's choice is compared with the fallback rule's choice, with the
library's own default (the tree rooted at the mode that cpd_als builds, default
tile) and with the fastest candidate.  Timings are live, on the kernels of
this build."""
import numpy as np
import pytest
import torch

from paper_1812_05961_amd import selector_train as st
from paper_1812_05961_amd import synth

pytestmark = pytest.mark.gpu

# held-out seeds (training used 0..1599) whose tensors have 0.5M..8M nonzeros
HELD_OUT = [s for s in range(1600, 2000)
            if 5e5 <= synth.selector_spec(s)["nnz"] <= 8e6][:8]


def test_network_beats_the_fallback_and_is_near_the_best():
    from paper_1812_05961_amd import cpd
    cpd.lib()
    params, hidden = st.load_params()
    ratio_net, ratio_heur, ratio_rooted = [], [], []
    for seed in HELD_OUT:
        spec = synth.selector_spec(seed)
        x = synth.selector_tensor(seed, device="cuda")
        stats, recs = st.time_tensor(x, spec["rank"], seed)
        s = cpd.tensor_stats(x.inds.to(torch.int32), x.dims)
        for r in recs:
            ch, _ = cpd.select(s, spec["rank"], r["mode"], params=params, hidden=hidden)
            pick = r["cands"].index(ch.as_dict(x.nmodes))
            ms = np.asarray(r["ms"])
            ratio_net.append(ms[pick] / ms.min())
            ratio_heur.append(ms[r["heur"]] / ms.min())
            ratio_rooted.append(ms[r["rooted"]] / ms.min())
        del x
    net, heur, rooted = np.array(ratio_net), np.array(ratio_heur), np.array(ratio_rooted)
    g_net = float(np.exp(np.log(net).mean()))
    g_heur = float(np.exp(np.log(heur).mean()))
    g_rooted = float(np.exp(np.log(rooted).mean()))
    print("cases %d: network/best geomean %.3f, fallback/best %.3f, rooted default/best %.3f, "
          "network within 10%%: %.2f" % (len(net), g_net, g_heur, g_rooted, float((net <= 1.10).mean())))
    assert len(net) >= 20
    # the network's choices run within 10% of the exhaustive best on average
    assert g_net <= 1.10, g_net
    # clearly faster than the fallback rule's
    assert g_heur / g_net >= 1.5, (g_heur, g_net)
    # and no slower than the library's own default layout
    assert g_net <= g_rooted, (g_net, g_rooted)
