"""The learned localiser's stored training and held-out evaluation (CPU only).

paper_2511_21647_amd/weights/ holds the weights trained by the library's own
kernels on simulated paper-scale ensembles 0..199 (MB counts drawn per ensemble
in [500, 8000]) and their evaluation on the 20 held-out ensembles 10000..10019,
scored by one-to-one matching within 0.5 px.  These tests tie the record to
that protocol and state the accuracy targets: the CNN must improve on NCC
against the truth, and the two stricter targets (recall of NCC's detections at
least 0.95, RMS error at most 0.1 px) are recorded as not met, with the
measured values in the failure message.  A second record scores the same
weights on the slab planes of the P = 8 sub-block form (35 slabs per
orientation, held-out ensembles 10000..10003), whose images hold a 35th of
the MBs each; there NCC's frame-relative intensity threshold passes many noise
peaks, so NCC is a weak reference, and the CNN is held to beating it against
the truth."""
import json
import os

import numpy as np
import pytest

W = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2511_21647_amd",
                 "weights")


def _load():
    with open(os.path.join(W, "cnn_paper_eval.json")) as fh:
        ev = json.load(fh)
    with open(os.path.join(W, "cnn_paper_train.json")) as fh:
        tr = json.load(fh)
    return ev, tr


def _load_slabs():
    with open(os.path.join(W, "cnn_paper_eval_slabs.json")) as fh:
        return json.load(fh)


def _pooled(ev, get):
    n_det = sum(get(r)["n_det"] for r in ev)
    n_ref = sum(get(r)["n_ref"] for r in ev)
    n_match = sum(get(r)["n_match"] for r in ev)
    sq = sum(get(r)["rms_px"] ** 2 * get(r)["n_match"] for r in ev if get(r)["n_match"])
    return {"recall": n_match / n_ref, "precision": n_match / n_det, "rms_px": float(np.sqrt(sq / n_match))}


def test_protocol():
    ev, tr = _load()
    assert tr["ensembles"] == 200 and len(tr["history"]) == 200
    train_ids = {h["ensemble"] for h in tr["history"]}
    assert train_ids == set(range(200))
    held = [r["ensemble"] for r in ev]
    assert held == list(range(10000, 10020))
    assert not set(held) & train_ids
    assert len({r["n_mb"] for r in ev}) > 10          # densities spread over the range


def test_cnn_improves_on_ncc_against_truth():
    """At some decode threshold the CNN finds more true MBs than NCC with a
    higher precision."""
    ev, _ = _load()
    ncc = _pooled(ev, lambda r: r["ncc_vs_truth"])
    better = []
    for thr in ev[0]["cnn"]:
        c = _pooled(ev, lambda r: r["cnn"][thr]["vs_truth"])
        if c["recall"] > ncc["recall"] and c["precision"] > ncc["precision"]:
            better.append((thr, round(c["recall"], 3), round(c["precision"], 3)))
    assert better, ncc


@pytest.mark.xfail(strict=True, reason="target not met: the CNN recovers at most about 0.60 of NCC's "
                                       "detections (0.75 of NCC's true ones) on the held-out ensembles")
def test_recall_of_ncc_target():
    ev, _ = _load()
    best = max(_pooled(ev, lambda r: r["cnn"][thr]["vs_ncc"])["recall"] for thr in ev[0]["cnn"])
    assert best >= 0.95, best


@pytest.mark.xfail(strict=True, reason="target not met: RMS error against the truth is 0.21-0.28 px "
                                       "for the CNN and 0.30 px for NCC at these MB densities")
def test_rms_target():
    ev, _ = _load()
    best = min(_pooled(ev, lambda r: r["cnn"][thr]["vs_truth"])["rms_px"] for thr in ev[0]["cnn"])
    assert best <= 0.1, best


def test_slab_protocol():
    ev, tr = _load()
    sl = _load_slabs()
    train_ids = {h["ensemble"] for h in tr["history"]}
    assert [r["ensemble"] for r in sl] == list(range(10000, 10004))
    assert not {r["ensemble"] for r in sl} & train_ids
    # the same held-out media as the full-plane record (same MB counts)
    assert [r["n_mb"] for r in sl] == [r["n_mb"] for r in ev[:4]]
    # each MB lies in one slab per orientation: the slab truth counts every MB of
    # the grid once per orientation and frame, like the two full planes
    for r, f in zip(sl, ev[:4]):
        assert r["ncc_vs_truth"]["n_ref"] == f["ncc_vs_truth"]["n_ref"]


def test_cnn_improves_on_ncc_on_slab_planes():
    """On the slab planes too some decode threshold finds more true MBs than NCC
    with a higher precision."""
    sl = _load_slabs()
    ncc = _pooled(sl, lambda r: r["ncc_vs_truth"])
    better = []
    for thr in sl[0]["cnn"]:
        if any(r["cnn"][thr].get("overflow") for r in sl):
            continue
        c = _pooled(sl, lambda r: r["cnn"][thr]["vs_truth"])
        if c["recall"] > ncc["recall"] and c["precision"] > ncc["precision"]:
            better.append((thr, round(c["recall"], 3), round(c["precision"], 3)))
    assert better, ncc
