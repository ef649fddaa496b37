"""Host-side logic of the MLMC drivers, on the CPU: the per-sample re-queue
of failed samples (with a stand-in for the batched solver) and the
append-only JSONL journal that the adaptive driver resumes from."""
import json

import pytest

import workloads as W


@pytest.fixture(scope="module")
def mods():
    torch = pytest.importorskip("torch")
    from paper_2212_04415_amd import beam as B
    from paper_2212_04415_amd import mlmc as PM
    from paper_2212_04415_amd import pd
    return torch, B, PM, pd


def fake_items(torch, B):
    lv = W.level(0, fracture=True)
    s0 = torch.arange(6 * 4, dtype=torch.float64).reshape(6, 4)
    c = 10.0 + s0
    return [B.BatchItem(None, B.make_params(lv), 6, s0, c), B.BatchItem(None, B.make_params(lv), 2, s0[:2].clone())]


def test_failed_samples_are_rerun_in_fp64_and_merged(mods):
    """Samples 2 and 5 of item 0 fail: one more batch runs exactly those two
    field rows with the item's parameters at FP64, and their results take
    the failed ones' places; item 1, which did not fail, is not re-run."""
    torch, B, PM, pd = mods
    items = fake_items(torch, B)
    calls = []

    def run(its, stream=None):
        calls.append(its)
        outs = []
        for k, it in enumerate(its):
            n = it.n_samples
            Q = torch.arange(n, dtype=torch.float64) + 100.0 * len(calls)
            st = torch.zeros(n, dtype=torch.int32)
            if len(calls) == 1 and k == 0:
                st[2], st[5] = pd.PD_ENONFINITE, pd.PD_EUNSTABLE
            outs.append((Q, torch.arange(n, dtype=torch.int64), st))
        return outs

    outs, requeued = PM.run_batch_requeue(items, run=run)
    assert requeued == [(0, 2), (0, 5)]
    assert len(calls) == 2 and len(calls[1]) == 1
    retry = calls[1][0]
    assert retry.n_samples == 2 and retry.params.precision == pd.PD_FP64
    assert items[0].params.precision == pd.PD_FP32          # the caller's block is untouched
    assert (retry.params.dt, retry.params.n_steps) == (items[0].params.dt, items[0].params.n_steps)
    assert torch.equal(retry.s0, items[0].s0[[2, 5]]) and torch.equal(retry.c, items[0].c[[2, 5]])
    assert retry.gf is None
    Q, ns, st = outs[0]
    assert Q.tolist() == [100.0, 101.0, 200.0, 103.0, 104.0, 201.0]
    assert ns.tolist() == [0, 1, 0, 3, 4, 1] and st.tolist() == [0] * 6
    assert outs[1][0].tolist() == [100.0, 101.0]


def test_a_sample_that_fails_again_is_reported(mods):
    torch, B, PM, pd = mods
    items = fake_items(torch, B)

    def run(its, stream=None):
        outs = []
        for it in its:
            st = torch.zeros(it.n_samples, dtype=torch.int32)
            st[0] = pd.PD_ENONFINITE
            outs.append((torch.zeros(it.n_samples, dtype=torch.float64),
                         torch.zeros(it.n_samples, dtype=torch.int64), st))
        return outs

    with pytest.raises(PM.SampleFailure) as ei:
        PM.run_batch_requeue(items, run=run)
    assert ei.value.failed == [(0, 0, pd.PD_ENONFINITE), (1, 0, pd.PD_ENONFINITE)]


def test_journal_reader_drops_a_torn_line_and_checks_the_header(mods, tmp_path):
    torch, B, PM, pd = mods
    header = dict(kind="header", tag={"seed": 3}, costs=[1.0, 8.0], dofs=[10.0, 80.0], eps=1.0, n_warm=4)
    path = tmp_path / "j.jsonl"
    recs = [header, dict(level=0, i=0, q_f=1.5, q_c=None, cost=1.0),
            dict(level=1, i=0, q_f=2.25, q_c=-0.1, cost=8.0)]
    whole = "".join(json.dumps(r) + "\n" for r in recs)
    path.write_text(whole + '{"level": 1, "i": 1, "q_f": 3.')
    got = PM._read_journal(str(path), header)
    assert got == {(0, 0): (1.5, None), (1, 0): (2.25, -0.1)}
    assert path.read_text() == whole                    # the torn tail is cut
    path.write_text(whole + '{"level": 1, "i": 1\n')    # a torn line that did get its newline
    assert PM._read_journal(str(path), header) == got and path.read_text() == whole
    with pytest.raises(ValueError, match="another configuration"):
        PM._read_journal(str(path), dict(header, eps=2.0))
    path.write_text(whole + "garbage\n" + json.dumps(recs[1]) + "\n")
    with pytest.raises(ValueError, match="not JSON"):
        PM._read_journal(str(path), header)
    assert PM._read_journal(str(tmp_path / "absent.jsonl"), header) == {}
