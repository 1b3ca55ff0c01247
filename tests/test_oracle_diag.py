"""Pins for the oracle's error-class diagnostics (Sec. II-C): the decision
hash keys against SplitMix64's published outputs, the recorded hash against
the decided message and its CRC, the ring order of the history, and the
classification on hand-built histories whose class and period are known."""
import json
import os

import numpy as np
import pytest

import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "published_constants.json")))


def _zobrist(keys, bits):
    h = 0
    for k, b in zip(keys, bits):
        if b:
            h ^= k
    return h


def test_key_zero_is_splitmix64_first_output(orc):
    # key(j) is the first SplitMix64 output from state j; state 0 is printed
    want = int(GOLD["splitmix64_seed0"]["outputs"][0], 16)
    assert orc.decision_key(0) == want


def test_keys_are_first_outputs_of_shifted_states(orc):
    # the k-th SplitMix64 output from state 0 is the first output from state
    # (k-1) * golden: the published second and third outputs pin the state
    # update that key(j) relies on; keys of distinct rows differ
    outs = [int(v, 16) for v in GOLD["splitmix64_seed0"]["outputs"]]
    g = 0x9E3779B97F4A7C15
    assert orc.splitmix64_stream(g, 1)[0] == outs[1]
    assert orc.splitmix64_stream((2 * g) % 2**64, 1)[0] == outs[2]
    assert all(orc.decision_key(j) == orc.splitmix64_stream(j, 1)[0] for j in (1, 7, 1023, 4095))
    assert len({orc.decision_key(j) for j in range(4096)}) == 4096


@pytest.mark.parametrize("N,K,cw,poly", [(64, 40, 8, 0x07), (256, 144, 16, 0x1021)])
def test_last_hash_of_an_accepted_frame_is_its_decided_word(orc, N, K, cw, poly):
    # a frame stopped by the CRC test has u on the information set equal to
    # its decided message followed by the message's CRC; the last recorded
    # hash must be the xor of the keys of that word's ones
    code = orc.construct(N, K, 2.0, cw, poly)
    F = 60
    msg = synth.message_bits(5, F, code.K_msg)
    _, x = orc.encode(code, msg)
    llr = synth.awgn_llr(x, 2.5, code.K_msg, seed=5)
    H = 8
    res, hist = orc.decode_trace(code, llr, orc.DecodeParams(max_iter=30, stop=orc.STOP_CRC), H,
                                 threads=4)
    keys = [orc.decision_key(int(j)) for j in code.info_idx]
    checked = 0
    for f in range(F):
        if not res.ok[f]:
            continue
        c = orc.crc(res.msg_hat[f], cw, poly)
        crc_bits = [(c >> (cw - 1 - t)) & 1 for t in range(cw)]
        word = list(res.msg_hat[f]) + crc_bits
        assert int(hist[f, (res.iters[f] - 1) % H]) == _zobrist(keys, word), f
        checked += 1
    assert checked > F // 2


def test_noiseless_frames_hash_their_word_every_iteration(orc):
    N, K = 128, 64
    code = orc.construct(N, K, 2.0, 8, 0x07)
    msg = synth.message_bits(9, 6, code.K_msg)
    u, x = orc.encode(code, msg)
    llr = np.where(x == 0, 20.0, -20.0).astype(np.float32)
    res, hist = orc.decode_trace(code, llr, orc.DecodeParams(max_iter=7, stop=orc.STOP_NONE), 16)
    for f in range(6):
        want = _zobrist([orc.decision_key(j) for j in range(N)], u[f])
        assert np.all(hist[f, :7] == want)
        assert np.all(hist[f, 7:] == 0)      # iterations never reached
    cls, per = orc.classify(res.msg_hat, msg, res.ok, res.iters, hist)
    assert np.all(cls == orc.CORRECT) and np.all(per == 1)


def test_history_ring_keeps_the_last_H_iterations(orc):
    code = orc.construct(128, 72, 1.5, 8, 0x07)
    msg = synth.message_bits(3, 40, code.K_msg)
    _, x = orc.encode(code, msg)
    llr = synth.awgn_llr(x, 0.5, code.K_msg, seed=3)
    p = orc.DecodeParams(max_iter=23, stop=orc.STOP_NONE)
    r64, h64 = orc.decode_trace(code, llr, p, 64, threads=4)
    r5, h5 = orc.decode_trace(code, llr, p, 5, threads=4)
    assert np.array_equal(r64.msg_hat, r5.msg_hat)
    for it in range(19, 24):                 # iterations 19..23 live in the 5-ring
        assert np.array_equal(h5[:, (it - 1) % 5], h64[:, it - 1])
    ref = orc.decode(code, llr, p, threads=4)
    assert np.array_equal(ref.msg_hat, r64.msg_hat) and np.array_equal(ref.iters, r64.iters)


def _ring(seq, iters, H, junk=0xDEAD):
    """Place seq (oldest first, the last len(seq) iterations) in an H-ring."""
    row = np.full(H, junk, np.uint64)
    W = len(seq)
    for i, v in enumerate(seq):
        row[(iters - W + i) % H] = v
    return row


@pytest.mark.parametrize("seq,iters,ok,wrong,cls,per", [
    ([5, 5, 5, 5, 5, 5, 5, 5], 70, 0, 1, 1, 1),          # stationary wrong decisions
    ([1, 2, 1, 2, 1, 2, 1, 2], 70, 0, 1, 2, 2),          # two-word cycle
    ([1, 2, 3, 1, 2, 3, 1, 2], 70, 0, 1, 2, 3),          # three-word cycle, length not a multiple
    ([1, 2, 3, 4, 5, 6, 7, 8], 70, 0, 1, 3, 0),          # no repetition
    ([1, 2, 1, 2, 1, 2, 1, 3], 70, 0, 1, 3, 0),          # a cycle broken by the last iteration
    ([9, 8, 7, 6, 5, 4, 3, 3], 70, 0, 1, 3, 0),          # settles only in the last two: p = 1 needs all
    ([1, 2, 3, 4, 5, 6, 7, 8], 70, 1, 1, 1, 0),          # the stop test accepted a wrong word
    ([1, 2, 3, 4, 5, 6, 7, 8], 70, 0, 0, 0, 0),          # correct whatever the history
    ([4], 1, 0, 1, 3, 0),                                # one iteration: no period can show
    ([4, 4], 2, 0, 1, 1, 1),
    ([4, 6, 4], 3, 0, 1, 3, 0),                          # period 2 needs four samples
])
def test_classification_of_hand_built_histories(orc, seq, iters, ok, wrong, cls, per):
    H = 8
    K = 5
    msg = np.zeros((1, K), np.uint8)
    hat = msg.copy()
    hat[0, 2] ^= wrong
    hist = _ring(seq, iters, H)[None, :]
    c, p = orc.classify(hat, msg, np.array([ok], np.uint8), np.array([iters], np.int32), hist)
    assert (int(c[0]), int(p[0])) == (cls, per)


def test_classification_reads_the_ring_oldest_first(orc):
    # a period-3 sequence of length 8 stays periodic only in its own order;
    # any rotation puts a seam inside the window
    H, iters = 8, 70
    seq = [1, 2, 3, 1, 2, 3, 1, 2]
    msg = np.zeros((1, 4), np.uint8)
    hat = msg.copy()
    hat[0, 0] = 1
    for rot in range(H):
        row = np.roll(_ring(seq, iters, H), rot)[None, :]
        c, p = orc.classify(hat, msg, np.zeros(1, np.uint8), np.array([iters], np.int32), row)
        assert (int(c[0]), int(p[0])) == ((2, 3) if rot == 0 else (3, 0)), rot


def test_classes_of_a_decoded_batch_are_consistent(orc):
    code = orc.construct(256, 128, 2.0, 16, 0x1021)
    F = 200
    msg = synth.message_bits(13, F, code.K_msg)
    _, x = orc.encode(code, msg)
    llr = synth.awgn_llr(x, 1.0, code.K_msg, seed=13)
    res, hist = orc.decode_trace(code, llr, orc.DecodeParams(max_iter=40, stop=orc.STOP_CRC), 16,
                                 threads=8)
    cls, per = orc.classify(res.msg_hat, msg, res.ok, res.iters, hist)
    wrong = (res.msg_hat != msg).any(1)
    assert np.array_equal(cls == orc.CORRECT, ~wrong)
    assert np.all(cls[wrong & (res.ok == 1)] == orc.FALSE_CONVERGED)
    assert np.all((per[cls == orc.OSCILLATION] >= 2))
    assert np.all(per[cls == orc.UNCONVERGED] == 0)
    assert wrong.sum() > 10 and len(set(cls[wrong].tolist())) >= 2
